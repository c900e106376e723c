// Locally low-rank proximal step (Sec. III-C, eqs. (20), (22), (23)).
//
// For every patch i the Casorati matrix P_i = Q_{q_i}(X) (p^2 x L) is thresholded:
//   P_i = U S V^H,  P'_i = U_r diag(max(sigma - tau, 0)) V_r^H  (at most r_cap values kept)
// computed without the L-sided vectors: with the Gram G_i = P_i P_i^H = U S^2 U^H,
//   P'_i = U_r diag(f) U_r^H P_i,   f_k = max(sigma_k - tau, 0) / sigma_k,   sigma_k = sqrt(lambda_k).
// Steps (kernels):
//   k_gram      G_i on MFMA (v_mfma_f32_16x16x4f32) from the real [Re P | Im P] blocks, FP32
//   k_tridiag   complex Householder reduction of G_i to a real symmetric tridiagonal T, in FP64
//   k_eig_val   all eigenvalues of T by Sturm bisection (one lane per eigenvalue), the nuclear
//               norm sum_k sigma_k, the r_cap largest eigenvalues and their factors f_k
//   k_eig_vec   eigenvectors of T for those with f_k > 0 by inverse iteration (thread per vector)
//   k_backxf    eigenvectors of G_i = Q D z (reflectors Q, phases D), clusters re-orthogonalised
//   k_coef      C_i = diag(f) U_r^H P_i  (r_cap x L per patch)
//   k_xupdate   X+ = (Z + k Q*(U_r C)) / (1 + k c), k = mu lam2 beta, c = patch coverage; a
//               16 x 16 pixel tile stages the C rows of the patches that cover it in LDS
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "patch.hpp"

namespace mrf {

constexpr int kMaxPP = 64;    // p^2 <= 64
constexpr int kMaxRllr = 16;

struct dcplx {
  double x, y;
};
__device__ inline dcplx dadd(dcplx a, dcplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline dcplx dsub(dcplx a, dcplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline dcplx dmul(dcplx a, dcplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline dcplx dconjmul(dcplx a, dcplx b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
__device__ inline dcplx dscale(dcplx a, double s) { return {a.x * s, a.y * s}; }

// Sum over the 64 lanes of a wave, returned in every lane; the whole wave must be active.
// Within each 16-lane row by DPP (quad permutes for xor 1 and xor 2, then row rotations by 4
// and 8), then the four row sums read with readlane, in a fixed order.
template <int CTRL>
__device__ inline double dpp64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  // every lane has a source lane under these controls, so no old value is needed
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false));
}
__device__ inline double row_sum16(double v) {
  v += dpp64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp64<0x124>(v);   // row_ror 4
  v += dpp64<0x128>(v);   // row_ror 8
  return v;
}
__device__ inline double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ inline double wave_sum(double v) {
  v = row_sum16(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}
// Two independent wave sums with their DPP steps interleaved (each in the order of wave_sum).
__device__ inline void wave_sum2(double& a, double& b) {
  a += dpp64<0xB1>(a);
  b += dpp64<0xB1>(b);
  a += dpp64<0x4E>(a);
  b += dpp64<0x4E>(b);
  a += dpp64<0x124>(a);
  b += dpp64<0x124>(b);
  a += dpp64<0x128>(a);
  b += dpp64<0x128>(b);
  a = (lane_value(a, 0) + lane_value(a, 16)) + (lane_value(a, 32) + lane_value(a, 48));
  b = (lane_value(b, 0) + lane_value(b, 16)) + (lane_value(b, 32) + lane_value(b, 48));
}

// Patch index of the b-th block, XCD-aware: blocks go to the 8 XCDs round-robin, and each XCD
// gets a contiguous band of patch rows so that overlapping patches share its L2.
__device__ inline int patch_of_block(int Np) {
  const int b = blockIdx.x;
  const int per = (Np + 7) / 8;
  const int i = (b & 7) * per + (b >> 3);
  return i < Np ? i : -1;
}
inline int patch_blocks(int Np) { return 8 * ((Np + 7) / 8); }

// ------------------------------------------------------------------ Gram on MFMA
typedef float f32x4 __attribute__((ext_vector_type(4)));

// G_i = P_i P_i^H, p^2 = PP, on the real parts: with P = Pr + i Pi,
//   Re G = Pr Pr^T + Pi Pi^T,   Im G = Pi Pr^T - Pr Pi^T.
// The 16 x 16 tiles (a, b) of the upper triangle are shared out over the block's waves; per
// group of 4 frames a lane reads one complex value of each operand from LDS and issues the four
// MFMAs of the tile's real and imaginary parts. The frame groups of a chunk are unrolled so that
// the LDS reads run ahead of the MFMAs. The kernel writes both triangles.
template <int PP>
struct GramCfg {
  static constexpr int NT = PP / 16;                 // tiles per side
  static constexpr int NUP = NT * (NT + 1) / 2;      // upper tiles
  static constexpr int NW = NUP >= 5 ? 5 : NUP;      // waves per block
  static constexpr int TPW = (NUP + NW - 1) / NW;    // tiles per wave
  static constexpr int NTHR = 64 * NW;
  static constexpr int FCH = 64;                     // frames per LDS chunk
  static constexpr int PER = (FCH * PP + NTHR - 1) / NTHR;
};
template <int PP>
__global__ __launch_bounds__(GramCfg<PP>::NTHR) void k_gram(const cf* __restrict__ X, PatchGeom g, int L,
                                                            cf* __restrict__ G) {
  typedef GramCfg<PP> C;
  constexpr int FCH = C::FCH, TPW = C::TPW, PER = C::PER, NTHR = C::NTHR;
  __shared__ cf P[FCH][PP];
  const int i = patch_of_block(g.Np);
  if (i < 0) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int oy = (i / g.n1) * g.s, ox = (i % g.n1) * g.s;
  const size_t NN = (size_t)g.N * g.N;
  static_assert(C::NUP % C::NW == 0, "every wave takes the same number of tiles");
  int ta[TPW], tb[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int u = w + q * C::NW, a = 0;
    while (u >= C::NT - a) {
      u -= C::NT - a;
      ++a;
    }
    ta[q] = a;
    tb[q] = a + u;
  }
  f32x4 accr[TPW], acci[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    accr[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    acci[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  cf nxt[PER];
  auto load = [&](int l0) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * NTHR, f = idx / PP, a = idx % PP;
      nxt[k] = idx < FCH * PP && l0 + f < L
                   ? X[(size_t)(l0 + f) * NN + (size_t)(oy + a / g.p) * g.N + ox + a % g.p]
                   : cf{0.f, 0.f};
    }
  };
  load(0);
  for (int l0 = 0; l0 < L; l0 += FCH) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * NTHR;
      if (idx < FCH * PP) P[idx / PP][idx % PP] = nxt[k];
    }
    lds_sync();
    if (l0 + FCH < L) load(l0 + FCH);   // in flight during this chunk's MFMAs
    // operands of frame group f0 + 4 are read while the MFMAs of group f0 run
    cf pa[TPW], pb[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      pa[q] = P[lane / 16][ta[q] * 16 + lane % 16];
      pb[q] = P[lane / 16][tb[q] * 16 + lane % 16];
    }
#pragma unroll
    for (int f0 = 0; f0 < FCH; f0 += 4) {
      cf na[TPW], nb[TPW];
      if (f0 + 4 < FCH) {
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
          na[q] = P[f0 + 4 + lane / 16][ta[q] * 16 + lane % 16];
          nb[q] = P[f0 + 4 + lane / 16][tb[q] * 16 + lane % 16];
        }
      }
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        accr[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[q].x, pb[q].x, accr[q], 0, 0, 0);
        acci[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[q].y, pb[q].x, acci[q], 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        accr[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[q].y, pb[q].y, accr[q], 0, 0, 0);
        acci[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(-pa[q].x, pb[q].y, acci[q], 0, 0, 0);
      }
      if (f0 + 4 < FCH) {
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
          pa[q] = na[q];
          pb[q] = nb[q];
        }
      }
    }
    lds_sync();
  }
  cf* Gi = G + (size_t)i * PP * PP;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int a = ta[q] * 16 + 4 * (lane / 16) + e, b = tb[q] * 16 + lane % 16;
      if (ta[q] == tb[q] && a > b) continue;   // diagonal tiles: the upper half writes both halves
      const float vi = a == b ? 0.f : acci[q][e];
      Gi[(size_t)a * PP + b] = cf{accr[q][e], vi};
      Gi[(size_t)b * PP + a] = cf{accr[q][e], -vi};
    }
  }
}
// Cell-pair form for 8 x 8 patches at stride 4 (each patch = 2 x 2 cells of 4 x 4 pixels). Every
// 16 x 16 block of a patch Gram is a cell-pair product C(a, b) = sum_f x_a(f) x_b(f)^H of the
// two cells' pixels, and neighbouring patches share these blocks, so each distinct pair is formed
// once: per cell a, the five blocks D = C(a, a), H = C(a, a + (0, 1)), V = C(a, a + (1, 0)),
// DR = C(a, a + (1, 1)), DL = C(a, a + (1, -1)); every other pair inside a patch is the
// conjugate transpose of one of these. Cb[cell][type][u][v] with u, v the raster index inside the
// 4 x 4 cell. A block takes kGcW consecutive cells of one cell row, one wave per cell; the
// block's frames are staged in LDS as the 2 cell rows x (kGcW + 2) cells that its five
// products touch.
constexpr int kGcW = 4;    // cells per block
constexpr int kGcF = 16;   // frames per LDS chunk
constexpr int kGcPer = kGcF * 2 * (kGcW + 2) * 16 / (64 * kGcW);   // staged values per thread
static_assert(kGcF * 2 * (kGcW + 2) * 16 % (64 * kGcW) == 0, "whole chunks per thread");
__global__ __launch_bounds__(64 * kGcW, 3) void k_gram_cells(const cf* __restrict__ X, int N, int nc, int L,
                                                          cf* __restrict__ Cb) {
  constexpr int SW = kGcW + 2, RW = 4 * SW;   // cells per staged row, pixels per staged image row
  __shared__ cf S[kGcF][2][SW][16];
  const int nstrip = (nc + kGcW - 1) / kGcW, nblk = nc * nstrip;
  const int per = (nblk + 7) / 8;
  const int q = (blockIdx.x & 7) * per + (blockIdx.x >> 3);   // XCD x: a band of cell rows
  if (q >= nblk) return;
  const int cy = q / nstrip, cx0 = (q % nstrip) * kGcW;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int cx = cx0 + w;
  const bool vD = cx < nc, vH = vD && cx + 1 < nc, vV = vD && cy + 1 < nc, vDR = vH && vV, vDL = vV && cx >= 1;
  const size_t NN = (size_t)N * N;
  f32x4 accr[5], acci[5];
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    accr[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    acci[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // element k of this thread: frame f = e / (8 RW) of the chunk, staged image row r8, column xr;
  // its offset inside a frame-chunk of X (32-bit: < kGcF N^2), or -1 outside the image
  int off[kGcPer];
#pragma unroll
  for (int k = 0; k < kGcPer; ++k) {
    const int e = tid + k * 64 * kGcW;
    const int f = e / (8 * RW), rem = e % (8 * RW), r8 = rem / RW, xr = rem % RW;
    const int y = 4 * cy + r8, x = 4 * (cx0 - 1) + xr;
    off[k] = y < N && x >= 0 && x < N ? f * N * N + y * N + x : -1;
  }
  cf nxt[kGcPer];
  auto load = [&](int l0) {
    const cf* Xc = X + (size_t)l0 * NN;
#pragma unroll
    for (int k = 0; k < kGcPer; ++k) {
      const int f = (tid + k * 64 * kGcW) / (8 * RW);
      nxt[k] = off[k] >= 0 && l0 + f < L ? Xc[off[k]] : cf{0.f, 0.f};
    }
  };
  load(0);
  for (int l0 = 0; l0 < L; l0 += kGcF) {
#pragma unroll
    for (int k = 0; k < kGcPer; ++k) {
      const int e = tid + k * 64 * kGcW;
      const int f = e / (8 * RW), rem = e % (8 * RW), r8 = rem / RW, xr = rem % RW;
      S[f][r8 >> 2][xr >> 2][(r8 & 3) * 4 + (xr & 3)] = nxt[k];
    }
    lds_sync();
    if (l0 + kGcF < L) load(l0 + kGcF);   // in flight during this chunk's MFMAs
    if (vD) {
#pragma unroll 2
      for (int f0 = 0; f0 < kGcF; f0 += 4) {
        const int fr = f0 + (lane >> 4), px = lane & 15;
        const cf pa = S[fr][0][w + 1][px];
        const cf pb[5] = {pa, S[fr][0][w + 2][px], S[fr][1][w + 1][px], S[fr][1][w + 2][px], S[fr][1][w][px]};
        const bool on[5] = {true, vH, vV, vDR, vDL};
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          if (!on[t]) continue;
          accr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa.x, pb[t].x, accr[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa.y, pb[t].x, acci[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          if (!on[t]) continue;
          accr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa.y, pb[t].y, accr[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-pa.x, pb[t].y, acci[t], 0, 0, 0);
        }
      }
    }
    lds_sync();
  }
  const bool on[5] = {vD, vH, vV, vDR, vDL};
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    if (!on[t]) continue;
    cf* o = Cb + ((size_t)(cy * nc + cx) * 5 + t) * 256;
#pragma unroll
    for (int e = 0; e < 4; ++e) o[(4 * (lane >> 4) + e) * 16 + (lane & 15)] = cf{accr[t][e], acci[t][e]};
  }
}
inline bool gram_cells_ok(const PatchGeom& g) { return g.p == 8 && g.s == 4 && g.nc >= 2; }
inline int gram_cells_blocks(const PatchGeom& g) {
  const int nblk = g.nc * ((g.nc + kGcW - 1) / kGcW);
  return 8 * ((nblk + 7) / 8);
}

__global__ __launch_bounds__(256) void k_gram_small(const cf* __restrict__ X, PatchGeom g, int L, cf* __restrict__ G) {
  const int i = patch_of_block(g.Np);
  if (i < 0) return;
  const int PP = g.p * g.p;
  const int t = threadIdx.x;
  if (t >= PP * PP) return;
  const int a = t / PP, b = t % PP;
  const int oy = (i / g.n1) * g.s, ox = (i % g.n1) * g.s;
  const size_t NN = (size_t)g.N * g.N;
  const size_t pa = (size_t)(oy + a / g.p) * g.N + ox + a % g.p, pb = (size_t)(oy + b / g.p) * g.N + ox + b % g.p;
  float re = 0.f, im = 0.f;
  for (int l = 0; l < L; ++l) {
    const cf u = X[(size_t)l * NN + pa], v = X[(size_t)l * NN + pb];
    re += u.x * v.x + u.y * v.y;   // u conj(v)
    im += u.y * v.x - u.x * v.y;
  }
  G[(size_t)i * PP * PP + t] = cf{re, im};
}

// ------------------------------------------------------------------ FP64 Householder
// One 4-wave block per patch; A (n x n, Hermitian, FP64) lives in registers: lane r of wave w
// holds A[r][c] for the 16 columns c = w (mod 4). For k = 0 .. n-3:
//   x = A[k+1:, k], alpha = ||x||, phase = x0/|x0|, beta = -phase alpha, v = x - beta e1,
//   tau = 1 / (alpha (alpha + |x0|)) so that H = I - tau v v^H maps x to beta e1;
//   p = tau A22 v, K = tau/2 v^H p, w = p - K v, A22 -= v w^H + w v^H.
// Each wave forms its part of A22 v, the parts meet in LDS, and every wave then computes p, K
// and w itself and updates its columns; the wave that owns column k+1 forms the next reflector.
// Two block barriers per column. The reflectors are written out (v, tau); T has diagonal d and
// sub-diagonal e (complex), then the phases D make it real: D_0 = 1, D_{k+1} = D_k e_k / |e_k|,
// e_k -> |e_k|.
constexpr int kTdW = 4;            // waves per patch (measured faster than 2 or 8)
constexpr int kTdJ = kMaxPP / kTdW;   // columns per thread
constexpr int kTdG = 4;               // columns per guarded group of the update
// a[j] for a run-time j, as a masked sum so that the array stays in registers
__device__ inline dcplx pick(const dcplx (&a)[kTdJ], int j) {
  double xr = 0.0, xi = 0.0;
#pragma unroll
  for (int q = 0; q < kTdJ; ++q) {
    const double m = q == j ? 1.0 : 0.0;
    xr = fma(m, a[q].x, xr);
    xi = fma(m, a[q].y, xi);
  }
  return dcplx{xr, xi};
}
__global__ __launch_bounds__(64 * kTdW) void k_tridiag(const cf* __restrict__ G, const cf* __restrict__ Cb, PatchGeom g,
                                                int Np, int n, double* __restrict__ dd, double* __restrict__ ee,
                                                dcplx* __restrict__ refl, double* __restrict__ rtau,
                                                dcplx* __restrict__ phase) {
  __shared__ dcplx vs[2][kMaxPP];    // reflector of the step, double-buffered by step parity
  __shared__ dcplx pw[kTdW][kMaxPP];    // per-wave parts of A22 v
  __shared__ dcplx wsw[kTdW][kMaxPP];   // each wave's copy of w
  __shared__ dcplx es[kMaxPP];
  __shared__ double taus[2];
  const int i = patch_of_block(Np);
  if (i < 0) return;
  const int t = threadIdx.x, w = t >> 6, r = t & 63;
  const cf* Gi = G + (size_t)i * n * n;
  dcplx* Ri = refl + (size_t)i * n * n;     // reflector k stored in row k (entries k+1 .. n-1)
  dcplx a[kTdJ];
  if (Cb) {
    // Gram from cell-pair blocks (8 x 8 patch = cells 0 1 / 2 3): slots 0-3 the diagonal blocks
    // of cells 0-3, then H of cells 0 and 2, V of cells 0 and 1, DR of cell 0, DL of cell 1. A pair
    // (alpha, beta) with alpha < beta is stored as is, the reverse pair as its conjugate transpose;
    // inside a diagonal block only u <= v is read, so A is exactly Hermitian.
    __shared__ cf cblk[10][256];
    const int py = i / g.n1, px = i % g.n1, nc = g.nc;
    for (int e = t; e < 10 * 256; e += 64 * kTdW) {
      const int sl = e >> 8, o = e & 255;
      int cell, ty;
      if (sl < 4) { cell = sl; ty = 0; }
      else if (sl < 6) { cell = 2 * (sl - 4); ty = 1; }
      else if (sl < 8) { cell = sl - 6; ty = 2; }
      else if (sl == 8) { cell = 0; ty = 3; }
      else { cell = 1; ty = 4; }
      const int gc = (py + (cell >> 1)) * nc + px + (cell & 1);
      cblk[sl][o] = Cb[((size_t)gc * 5 + ty) * 256 + o];
    }
    __syncthreads();
    constexpr int kSlot[4][4] = {{0, 4, 6, 8}, {4, 1, 9, 7}, {6, 9, 2, 5}, {8, 7, 5, 3}};
    const int ca = ((r >> 3) >> 2) * 2 + ((r & 7) >> 2), u = ((r >> 3) & 3) * 4 + (r & 3);
#pragma unroll
    for (int j = 0; j < kTdJ; ++j) {
      const int c = kTdW * j + w;
      const int cbt = ((c >> 3) >> 2) * 2 + ((c & 7) >> 2), v = ((c >> 3) & 3) * 4 + (c & 3);
      const int sl = kSlot[ca][cbt];
      const bool direct = ca < cbt || (ca == cbt && u <= v);
      const cf x = direct ? cblk[sl][u * 16 + v] : cblk[sl][v * 16 + u];
      a[j] = dcplx{x.x, direct ? (double)x.y : -(double)x.y};
      if (ca == cbt && u == v) a[j].y = 0.0;
    }
  } else {
#pragma unroll
    for (int j = 0; j < kTdJ; ++j) {
      const int c = kTdW * j + w;
      cf x = cf{0.f, 0.f};
      if (r < n && c < n) x = Gi[(size_t)c * n + r];   // A[r][c] = conj(G[c][r])
      a[j] = dcplx{x.x, -(double)x.y};
    }
  }
  // reflector of column k from this wave's lanes x = A[r][k]
  auto reflector = [&](int k, dcplx x, int buf) {
    const bool below = r > k && r < n;
    const double alpha = sqrt(wave_sum(below ? x.x * x.x + x.y * x.y : 0.0));
    const double x0r = __shfl(x.x, k + 1), x0i = __shfl(x.y, k + 1);
    const double ax0 = sqrt(x0r * x0r + x0i * x0i);
    const double phr = ax0 > 0 ? x0r / ax0 : 1.0, phi = ax0 > 0 ? x0i / ax0 : 0.0;
    const bool live = alpha > 0.0;
    const double tau = live ? 1.0 / (alpha * (alpha + ax0)) : 0.0;
    const double br = -alpha * phr, bi = -alpha * phi;   // beta
    const bool head = r == k + 1, keep = live && below;
    const double vr = keep ? (head ? x.x - br : x.x) : 0.0;
    const double vi = keep ? (head ? x.y - bi : x.y) : 0.0;
    vs[buf][r] = dcplx{vr, vi};
    if (r > k && r < n) Ri[(size_t)k * n + r] = dcplx{vr, vi};   // only the entries the back-transform reads
    if (r == 0) {
      rtau[(size_t)i * n + k] = tau;
      taus[buf] = tau;
      es[k] = dcplx{live ? br : x0r, live ? bi : x0i};
    }
  };
  if (n > 2 && w == 0) reflector(0, a[0], 0);
  __syncthreads();
  for (int k = 0; k < n - 2; ++k) {
    const int buf = k & 1;
    const double tau = taus[buf];
    const bool below = r > k && r < n;
    // Columns are visited in groups of kTdG from the block-uniform bounds jlo = (k + 1) / 4 and
    // jhi = (n - 1) / 4, which include every column k < c < n of every wave. A column c <= k or
    // c >= n that a group brings in adds exact zeros: v and w vanish outside (k, n).
    const int jlo = (k + 1) >> 2, jhi = (n - 1) >> 2;
    if (tau != 0.0) {   // uniform over the block
      // (A22 v)_r over this wave's columns, accumulated by FMAs into two partial sums
      dcplx pp[2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
      for (int j = 0; j < kTdJ; j += kTdG) {
        if (j + kTdG - 1 >= jlo && j <= jhi) {
#pragma unroll
          for (int h = 0; h < kTdG; ++h) {
            const dcplx vc = vs[buf][kTdW * (j + h) + w];
            dcplx& q = pp[h & 1];
            q.x = fma(a[j + h].x, vc.x, q.x);
            q.x = fma(-a[j + h].y, vc.y, q.x);
            q.y = fma(a[j + h].x, vc.y, q.y);
            q.y = fma(a[j + h].y, vc.x, q.y);
          }
        }
      }
      pw[w][r] = below ? dadd(pp[0], pp[1]) : dcplx{0.0, 0.0};
      __syncthreads();
      const dcplx v = vs[buf][r];
      dcplx ps;
      if constexpr (kTdW == 4) ps = dadd(dadd(pw[0][r], pw[1][r]), dadd(pw[2][r], pw[3][r]));
      else if constexpr (kTdW == 2) ps = dadd(pw[0][r], pw[1][r]);
      else if constexpr (kTdW == 8)
        ps = dadd(dadd(dadd(pw[0][r], pw[1][r]), dadd(pw[2][r], pw[3][r])),
                  dadd(dadd(pw[4][r], pw[5][r]), dadd(pw[6][r], pw[7][r])));
      else ps = pw[0][r];
      const dcplx pv = dscale(ps, tau);
      double kr = below ? v.x * pv.x + v.y * pv.y : 0.0;
      double ki = below ? v.x * pv.y - v.y * pv.x : 0.0;
      wave_sum2(kr, ki);
      const dcplx K = dscale(dcplx{kr, ki}, 0.5 * tau);
      const dcplx wr = below ? dsub(pv, dmul(K, v)) : dcplx{0.0, 0.0};
      wsw[w][r] = wr;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (below) {
        // A[r][c] -= v_r conj(w_c) + w_r conj(v_c), as four FMAs per component
#pragma unroll
        for (int j = 0; j < kTdJ; j += kTdG) {
          if (j + kTdG - 1 >= jlo && j <= jhi) {
#pragma unroll
            for (int h = 0; h < kTdG; ++h) {
              const int c = kTdW * (j + h) + w;
              const dcplx wc = wsw[w][c], vc = vs[buf][c];
              a[j + h].x = fma(-v.x, wc.x, a[j + h].x);
              a[j + h].x = fma(-v.y, wc.y, a[j + h].x);
              a[j + h].x = fma(-wr.x, vc.x, a[j + h].x);
              a[j + h].x = fma(-wr.y, vc.y, a[j + h].x);
              a[j + h].y = fma(-v.y, wc.x, a[j + h].y);
              a[j + h].y = fma(v.x, wc.y, a[j + h].y);
              a[j + h].y = fma(-wr.y, vc.x, a[j + h].y);
              a[j + h].y = fma(wr.x, vc.y, a[j + h].y);
            }
          }
        }
      }
    }
    if (k + 1 < n - 2) {
      if (w == (k + 1) % kTdW) reflector(k + 1, pick(a, (k + 1) / kTdW), buf ^ 1);
      __syncthreads();
    }
  }
  if (n >= 2 && w == (n - 2) % kTdW) {   // e_{n-2} = A[n-1][n-2]
    const dcplx x = pick(a, (n - 2) / kTdW);
    const dcplx y = dcplx{__shfl(x.x, n - 1), __shfl(x.y, n - 1)};
    if (r == 0) es[n - 2] = y;
  }
  if (r < n && w == r % kTdW) dd[(size_t)i * n + r] = pick(a, r / kTdW).x;
  __syncthreads();
  if (t == 0) {
    dcplx D{1.0, 0.0};
    phase[(size_t)i * n + 0] = D;
    for (int k = 0; k < n - 1; ++k) {
      const dcplx e = es[k];
      const double ae = sqrt(e.x * e.x + e.y * e.y);
      ee[(size_t)i * n + k] = ae;
      if (ae > 0.0) D = dmul(D, dcplx{e.x / ae, e.y / ae});
      phase[(size_t)i * n + k + 1] = D;
    }
    ee[(size_t)i * n + n - 1] = 0.0;
  }
}

// Number of eigenvalues of the symmetric tridiagonal (d, e^2) smaller than x, from the signs of
// the pivots q_k = (d_k - x) - e_{k-1}^2 / q_{k-1} of the LDL^T factorisation of T - x I. The
// matrix is scaled so that |d|, e^2 <= 1; a pivot smaller than pmin in magnitude is replaced by
// -pmin (a perturbation of d_k by at most pmin). 1/q comes from the hardware reciprocal (about 24
// correct bits) refined by one Newton step: measured on gfx950 within 11 ulp of the correctly
// rounded value, a relative perturbation of the pivot of about 2e-15, far below the 1e-10 (of the
// spectrum's span) resolution the bisection stops at.
constexpr double kPivMin = 1e-280;
__device__ inline double recip(double q) {
  const double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}
// After the guard a pivot is never zero or NaN, so q < 0 is its sign bit.
__device__ inline unsigned neg_bit(double q) { return (unsigned)__double2hiint(q) >> 31; }
__device__ inline int sturm_count(const double* d, const double* e2, int n, double x) {
  double q = d[0] - x;
  if (fabs(q) < kPivMin) q = -kPivMin;
  unsigned c = neg_bit(q);
  for (int k = 1; k < n; ++k) {
    q = (d[k] - x) - e2[k - 1] * recip(q);
    if (fabs(q) < kPivMin) q = -kPivMin;
    c += neg_bit(q);
  }
  return (int)c;
}

__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// One wave per patch: all n eigenvalues of T by Sturm bisection, lane j finding the j-th smallest.
// T is scaled by a power of two sc so that its Gershgorin disc fits in [-1, 1]. One multisection
// sweep (lane j counts at the j-th of 64 equispaced points) brackets every eigenvalue to 1/64 of
// the spectrum's span before the per-lane bisection. Outputs: the patch's nuclear norm
// sum_j sqrt(max(lambda_j, 0)), the rcap largest eigenvalues (descending) and their shrinkage
// factors f_k = (sigma_k - tau)_+ / sigma_k.
__global__ __launch_bounds__(64) void k_eig_val(const double* __restrict__ dd, const double* __restrict__ ee, int Np,
                                               int n, double tau_thr, int rcap, double* __restrict__ nuc,
                                               double* __restrict__ lamtop, float* __restrict__ fk,
                                               double* __restrict__ lam_out) {
  __shared__ double d[kMaxPP], e2[kMaxPP], lam[kMaxPP];
  __shared__ int cnt[64];
  const int i = patch_of_block(Np);
  if (i < 0) return;
  const int t = threadIdx.x;
  const double dt = t < n ? dd[(size_t)i * n + t] : 0.0;
  const double et = t < n - 1 ? fabs(ee[(size_t)i * n + t]) : 0.0;
  const double etm = __shfl_up(et, 1);
  const double rad = et + (t > 0 ? etm : 0.0);
  const double g_lo = wave_min(t < n ? dt - rad : DBL_MAX);
  const double g_hi = wave_max(t < n ? dt + rad : -DBL_MAX);
  const double gmax = fmax(fabs(g_lo), fabs(g_hi));
  const double sc = gmax > 0.0 ? ldexp(1.0, ilogb(gmax) + 1) : 1.0;   // power of two > gmax
  const double isc = 1.0 / sc;
  if (t < n) {
    d[t] = dt * isc;
    e2[t] = (et * isc) * (et * isc);
  }
  __syncthreads();
  double lo = g_lo * isc, hi = g_hi * isc;
  const double span = fmax(hi - lo, 1e-250);
  lo -= 1e-12 * span + 1e-250;
  hi += 1e-12 * span + 1e-250;
  // multisection: cnt[j] = number of eigenvalues below x_j = lo + (j + 1) (hi - lo) / 64
  const double h = (hi - lo) * (1.0 / 64.0);
  const double xj = t == 63 ? hi : lo + (t + 1) * h;
  cnt[t] = sturm_count(d, e2, n, xj);
  __syncthreads();
  int j = 0;
  while (j < 63 && cnt[j] <= t) ++j;
  double a = j == 0 ? lo : lo + j * h;
  double b = j == 63 ? hi : lo + (j + 1) * h;
  // bisection to 1e-10 of the span: lambda_t (ascending) lies in (a, b]. The Gram comes from FP32
  // products over L frames, whose entries are off by about sqrt(2L) 2^-24 of the largest
  // eigenvalue (3e-6 at L = 1000); a finer stop would resolve nothing of that matrix.
  const double tol = 1e-10 * span;
  for (int it = 0; it < 48; ++it) {
    const double m = 0.5 * (a + b);
    const bool done = m <= a || m >= b || b - a <= tol;
    if (__all(done)) break;
    if (!done) {
      if (t < n && sturm_count(d, e2, n, m) > t) b = m;
      else a = m;
    }
  }
  const double lt = 0.5 * (a + b) * sc;
  if (t < n) lam[t] = lt;
  const double tot = wave_sum(t < n ? sqrt(fmax(lt, 0.0)) : 0.0);
  if (t == 0) nuc[i] = tot;
  __syncthreads();
  if (t < rcap) {
    const double lk = t < n ? lam[n - 1 - t] : 0.0;
    const double sk = sqrt(fmax(lk, 0.0));
    const double f = sk > tau_thr ? (sk - tau_thr) / sk : 0.0;
    fk[(size_t)i * rcap + t] = (float)f;
    lamtop[(size_t)i * rcap + t] = lk;
    if (lam_out) lam_out[(size_t)i * rcap + t] = lk;
  }
}

// Eigenvectors of T for the rcap largest eigenvalues by inverse iteration, one thread per
// (patch, k). Each sweep factors T - lambda_k I = P L U (partial pivoting; a pivot below
// 1e-14 |T| is replaced by that bound) while it eliminates the right-hand side, then
// back-substitutes with U; three sweeps from a fixed start vector. Components with f_k = 0 get a
// zero vector. The thread's shifted T, U and right-hand side live in LDS, interleaved by thread.
constexpr int kEvT = 16;   // threads per block
__global__ __launch_bounds__(kEvT) void k_eig_vec(const double* __restrict__ dd, const double* __restrict__ ee,
                                                  const double* __restrict__ lamtop, const float* __restrict__ fk,
                                                  int Np, int n, int rcap, double* __restrict__ zvec) {
  __shared__ double ds[kMaxPP][kEvT], es[kMaxPP][kEvT];
  __shared__ double ui[kMaxPP][kEvT], u1[kMaxPP][kEvT], u2[kMaxPP][kEvT], y[kMaxPP][kEvT];
  const int t = threadIdx.x;
  const long gid = (long)blockIdx.x * kEvT + t;
  if (gid >= (long)Np * rcap) return;
  const int i = (int)(gid / rcap), k = (int)(gid % rcap);
  double* z = zvec + ((size_t)i * rcap + k) * n;
  if (k >= n || fk[(size_t)i * rcap + k] <= 0.f) {
    for (int q = 0; q < n; ++q) z[q] = 0.0;
    return;
  }
  const double* d = dd + (size_t)i * n;
  const double* e = ee + (size_t)i * n;
  const double lk = lamtop[(size_t)i * rcap + k];
  double tn = 0.0;
#pragma unroll 8
  for (int q = 0; q < n; ++q) {
    const double dq = d[q], eq = q < n - 1 ? e[q] : 0.0;
    ds[q][t] = dq - lk;
    es[q][t] = eq;
    tn = fmax(tn, fabs(dq) + 2.0 * fabs(eq));
    y[q][t] = 1.0 + 0.01 * ((q * 37 + k * 11) % 7);
  }
  const double eps = 1e-14 * tn + 1e-300;
  double scale = 1.0;
  for (int sweep = 0; sweep < 3; ++sweep) {
    // factor and eliminate: the partly reduced row q is (dcur, ecur) at columns (q, q + 1)
    double dcur = ds[0][t], ecur = es[0][t];
    double yc = y[0][t] * scale;
    for (int q = 0; q < n - 1; ++q) {
      const double sub = es[q][t];
      const double nd = ds[q + 1][t], ne = es[q + 1][t];
      const double yn = y[q + 1][t] * scale;
      if (fabs(dcur) >= fabs(sub)) {
        const double piv = fabs(dcur) < eps ? eps : dcur;
        const double rp = 1.0 / piv, ml = sub * rp;
        ui[q][t] = rp; u1[q][t] = ecur; u2[q][t] = 0.0;
        y[q][t] = yc;
        yc = yn - ml * yc;
        dcur = nd - ml * ecur;
        ecur = ne;
      } else {
        const double rp = 1.0 / sub, ml = dcur * rp;
        ui[q][t] = rp; u1[q][t] = nd; u2[q][t] = ne;
        y[q][t] = yn;
        yc = yc - ml * yn;
        dcur = ecur - ml * nd;
        ecur = -ml * ne;
      }
    }
    ui[n - 1][t] = 1.0 / (fabs(dcur) < eps ? eps : dcur);
    y[n - 1][t] = yc;
    // back substitution
    double y1 = 0.0, y2 = 0.0, nr = 0.0;
    for (int q = n - 1; q >= 0; --q) {
      const double v = (y[q][t] - u1[q][t] * y1 - u2[q][t] * y2) * ui[q][t];
      y[q][t] = v;
      nr += v * v;
      y2 = y1;
      y1 = v;
    }
    scale = 1.0 / sqrt(fmax(nr, 1e-300));
  }
  for (int q = 0; q < n; ++q) z[q] = y[q][t] * scale;
}

// The same inverse iteration for n = N known at compile time, with the thread's LU factors and
// right-hand side in registers (no LDS, so many threads per CU): the pivoting choice is a select
// rather than a branch, and the second superdiagonal of U is non-zero only where rows were
// swapped, where it equals the next off-diagonal of T (one bit per row records the swap). Same
// arithmetic as k_eig_vec.
template <int N>
__global__ __launch_bounds__(64) void k_eig_vec_reg(const double* __restrict__ dd, const double* __restrict__ ee,
                                                    const double* __restrict__ lamtop, const float* __restrict__ fk,
                                                    int Np, int rcap, double* __restrict__ zvec) {
  static_assert(N >= 3 && N <= 64, "register inverse iteration needs 3 <= n <= 64");
  const long gid = (long)blockIdx.x * 64 + threadIdx.x;
  if (gid >= (long)Np * rcap) return;
  const int i = (int)(gid / rcap), k = (int)(gid % rcap);
  double* z = zvec + ((size_t)i * rcap + k) * N;
  if (k >= N || fk[(size_t)i * rcap + k] <= 0.f) {
    for (int q = 0; q < N; ++q) z[q] = 0.0;
    return;
  }
  const double* d = dd + (size_t)i * N;
  const double* e = ee + (size_t)i * N;
  const double lk = lamtop[(size_t)i * rcap + k];
  double tn = 0.0;
#pragma unroll
  for (int q = 0; q < N; ++q) tn = fmax(tn, fabs(d[q]) + 2.0 * fabs(q < N - 1 ? e[q] : 0.0));
  const double eps = 1e-14 * tn + 1e-300;
  // T is re-read (from cache) one step ahead inside the sweeps: the empty asm statements with a
  // memory clobber keep the compiler from holding all of d and e in registers next to the three
  // n-long arrays below.
  asm volatile("" ::: "memory");
  double y[N], ui[N], u1[N];
#pragma unroll
  for (int q = 0; q < N; ++q) y[q] = 1.0 + 0.01 * ((q * 37 + k * 11) % 7);
  double scale = 1.0;
  for (int sweep = 0; sweep < 3; ++sweep) {
    unsigned long long swp = 0ull;
    double dcur = d[0] - lk, ecur = e[0];
    double yc = y[0] * scale;
    double eq = e[0], dq1 = d[1], eq1 = e[1];   // e[q], d[q+1], e[q+1] of step q
#pragma unroll
    for (int q = 0; q < N - 1; ++q) {
      const double dq2 = q + 2 < N ? d[q + 2] : 0.0, eq2 = q + 2 < N - 1 ? e[q + 2] : 0.0;
      asm volatile("" ::: "memory");
      const double sub = eq;
      const double nd = dq1 - lk, ne = q + 1 < N - 1 ? eq1 : 0.0;
      const double yn = y[q + 1] * scale;
      const bool sw = !(fabs(dcur) >= fabs(sub));
      const double piv = fabs(dcur) < eps ? eps : dcur;
      const double rp = 1.0 / (sw ? sub : piv);
      const double ml = (sw ? dcur : sub) * rp;
      ui[q] = rp;
      u1[q] = sw ? nd : ecur;
      const double ya = sw ? yc : yn, yb = sw ? yn : yc;
      y[q] = yb;
      yc = ya - ml * yb;
      const double da = sw ? ecur : nd, db = sw ? nd : ecur;
      dcur = da - ml * db;
      ecur = sw ? -ml * ne : ne;
      swp |= (unsigned long long)sw << q;
      eq = eq1;
      dq1 = dq2;
      eq1 = eq2;
    }
    ui[N - 1] = 1.0 / (fabs(dcur) < eps ? eps : dcur);
    double y1 = yc * ui[N - 1], y2 = 0.0;
    y[N - 1] = y1;
    double nr = y1 * y1;
    double en = 0.0;                              // e[q+1] of step q (0 for q = n - 2)
#pragma unroll
    for (int q = N - 2; q >= 0; --q) {
      const double ep = q >= 1 ? e[q] : 0.0;      // for step q - 1
      asm volatile("" ::: "memory");
      const double u2 = (swp >> q) & 1ull ? en : 0.0;
      const double v = (y[q] - u1[q] * y1 - u2 * y2) * ui[q];
      y[q] = v;
      nr += v * v;
      y2 = y1;
      y1 = v;
      en = ep;
    }
    scale = 1.0 / sqrt(fmax(nr, 1e-300));
  }
#pragma unroll
  for (int q = 0; q < N; ++q) z[q] = y[q] * scale;
}

// u_k = H_0 H_1 ... H_{n-3} D z_k for the rcap vectors. One block per patch with one wave per four
// vectors; the patch's reflectors (entries k+1 .. n-1 of row k) are read from cache, the next one
// while the current one is applied. Wave 0 first orthogonalises, in the tridiagonal basis, each
// vector against the earlier ones of its cluster (eigenvalues within 1e-6 of the largest; modified
// Gram-Schmidt). Then wave w back-transforms vectors k = 4 w + s, s = lane / 16: each vector lives
// in one 16-lane DPP row,
// lane l of the row holding rows l, l + 16, l + 32, l + 48, so the reflector's inner product with
// the vector is a 16-lane row sum. Stores U[i][k][a] (FP32); components with f_k = 0 (zero z) get
// zero vectors.
__global__ __launch_bounds__(256) void k_backxf(const double* __restrict__ zvec, const double* __restrict__ lamtop,
                                               const dcplx* __restrict__ refl, const double* __restrict__ rtau,
                                               const dcplx* __restrict__ phase, int Np, int n, int rcap,
                                               cf* __restrict__ U) {
  __shared__ double zs[kMaxRllr][kMaxPP];
  __shared__ double tau[kMaxPP];
  __shared__ int live[kMaxRllr];
  const int i = patch_of_block(Np);
  if (i < 0) return;
  const int nt = blockDim.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const dcplx* Ri = refl + (size_t)i * n * n;   // reflector j in row j, entries j+1 .. n-1 (read from cache)
  const int nref = n - 2 > 0 ? n - 2 : 0;
  if (t < n) tau[t] = t < nref ? rtau[(size_t)i * n + t] : 0.0;
  const int m = min(rcap, n);
  for (int idx = t; idx < m * kMaxPP; idx += nt) {
    const int k = idx / kMaxPP, q = idx % kMaxPP;
    zs[k][q] = q < n ? zvec[((size_t)i * rcap + k) * n + q] : 0.0;
  }
  __syncthreads();
  if (w == 0) {
    const double* lt = lamtop + (size_t)i * rcap;
    const double ctol = 1e-6 * fmax(fabs(lt[0]), 1e-300);
    for (int k = 0; k < m; ++k) {
      double z = zs[k][lane];
      const bool lv = wave_sum(z * z) != 0.0;
      if (lane == 0) live[k] = lv;
      if (!lv) continue;
      bool moved = false;
      for (int j = 0; j < k; ++j) {
        if (fabs(lt[k] - lt[j]) > ctol) continue;
        const double zj = zs[j][lane];
        z -= wave_sum(zj * z) * zj;
        moved = true;
      }
      if (moved) {
        z *= 1.0 / sqrt(fmax(wave_sum(z * z), 1e-300));
        zs[k][lane] = z;
      }
    }
  }
  __syncthreads();
  const int t16 = lane & 15, k = 4 * w + (lane >> 4);
  const bool on = k < m && live[k];
  dcplx u[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = t16 + 16 * a;
    u[a] = on && r < n ? dscale(phase[(size_t)i * n + r], zs[k][r]) : dcplx{0.0, 0.0};
  }
  if (__ballot(on) != 0ull) {
    // the next reflector's entries are loaded while this one is applied
    auto ldv = [&](int j, dcplx (&v)[4]) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int r = t16 + 16 * a;
        v[a] = j >= 0 && r > j && r < n ? Ri[(size_t)j * n + r] : dcplx{0.0, 0.0};
      }
    };
    dcplx vn[4];
    ldv(nref - 1, vn);
    for (int j = nref - 1; j >= 0; --j) {
      dcplx v[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) v[a] = vn[a];
      ldv(j - 1, vn);
      const double tj = tau[j];
      if (tj == 0.0) continue;
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        dr += v[a].x * u[a].x + v[a].y * u[a].y;
        di += v[a].x * u[a].y - v[a].y * u[a].x;
      }
      dr = row_sum16(dr);
      di = row_sum16(di);
      const dcplx gk = {tj * dr, tj * di};
#pragma unroll
      for (int a = 0; a < 4; ++a) u[a] = dsub(u[a], dmul(v[a], gk));
    }
  }
  if (k < m) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = t16 + 16 * a;
      if (r < n) U[((size_t)i * rcap + k) * n + r] = cf{(float)u[a].x, (float)u[a].y};
    }
  }
  if (w == 0)   // rank cap above the patch size: zero rows
    for (int kk = m; kk < rcap; ++kk)
      for (int r = lane; r < n; r += 64) U[((size_t)i * rcap + kk) * n + r] = cf{0.f, 0.f};
}

// C[i][k][l] = f_k sum_a conj(U[i][k][a]) X[l][pixel a of patch i] on MFMA: D (k x frames) =
// A (k x pixels) B (pixels x frames) with A = U^H held in registers (rows k >= rcap are zero) and
// B staged in LDS per chunk of 64 frames, read by the 4 waves one 16-frame tile each. Rows of the
// LDS chunk are padded by one value (row stride = 2 mod 32 banks), so the 16 frames read by a
// quarter-wave fall on distinct bank pairs.
template <int PP>
__global__ __launch_bounds__(256) void k_coef(const cf* __restrict__ X, const cf* __restrict__ U,
                                              const float* __restrict__ fk, PatchGeom g, int L, int rcap,
                                              cf* __restrict__ C) {
  constexpr int FCH = 64, PER = FCH * PP / 256, NA = PP / 4;
  __shared__ cf P[FCH][PP + 1];
  const int i = patch_of_block(g.Np);
  if (i < 0) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int oy = (i / g.n1) * g.s, ox = (i % g.n1) * g.s;
  const size_t NN = (size_t)g.N * g.N;
  // A[m][kk] = conj(U[k = m][a0 + kk]): lane supplies m = lane % 16, kk = lane / 16
  cf ua[NA];
  {
    const int k = lane % 16;
#pragma unroll
    for (int s = 0; s < NA; ++s)
      ua[s] = k < rcap ? U[((size_t)i * rcap + k) * PP + s * 4 + lane / 16] : cf{0.f, 0.f};
  }
  float fo[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = 4 * (lane / 16) + e;
    fo[e] = k < rcap ? fk[(size_t)i * rcap + k] : 0.f;
  }
  cf nxt[PER];
  auto load = [&](int l0) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * 256, f = idx / PP, a = idx % PP;
      nxt[k] = l0 + f < L ? X[(size_t)(l0 + f) * NN + (size_t)(oy + a / g.p) * g.N + ox + a % g.p] : cf{0.f, 0.f};
    }
  };
  load(0);
  for (int l0 = 0; l0 < L; l0 += FCH) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * 256;
      P[idx / PP][idx % PP] = nxt[k];
    }
    lds_sync();
    if (l0 + FCH < L) load(l0 + FCH);
    f32x4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NA; ++s) {
      const cf bv = P[w * 16 + lane % 16][s * 4 + lane / 16];
      dr = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[s].x, bv.x, dr, 0, 0, 0);
      dr = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[s].y, bv.y, dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[s].x, bv.y, di, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_16x16x4f32(-ua[s].y, bv.x, di, 0, 0, 0);
    }
    const int f = l0 + w * 16 + lane % 16;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * (lane / 16) + e;
      if (k < rcap && f < L) C[((size_t)i * rcap + k) * L + f] = cf{dr[e] * fo[e], di[e] * fo[e]};
    }
    lds_sync();
  }
}

// Any p^2 <= 64: block per patch, thread per frame.
// The same coefficients for 8 x 8 patches at stride 4, organised for reuse of X: a block takes 4
// neighbouring patches of one patch row (one wave each) and a chunk of kCsChunk frames (the
// patches' U is read once per chunk). Per 16 frames the block stages the 8 x 20 pixels its
// patches cover in LDS (frame stride 161 values: the 16 frames read by a quarter-wave fall on
// distinct bank pairs) and each wave forms its 16 x 16 tile on MFMA. Blocks are numbered chunk-major and dealt to the XCDs in contiguous ranges, so each
// XCD runs through all patch rows of its frames and consecutive rows find their shared pixels in
// its L2.
#ifndef MRF_CS_CHUNK
#define MRF_CS_CHUNK 256
#endif
constexpr int kCsF = 16, kCsChunk = MRF_CS_CHUNK, kCsW = 20, kCsFS = 8 * kCsW + 1;
constexpr int kCsPer = kCsF * 8 * kCsW / 256;   // staged values per thread
static_assert(kCsF * 8 * kCsW % 256 == 0, "whole stage per thread");
__global__ __launch_bounds__(256) void k_coef_strip(const cf* __restrict__ X, const cf* __restrict__ U,
                                                    const float* __restrict__ fk, PatchGeom g, int L, int rcap,
                                                    cf* __restrict__ C) {
  __shared__ cf S[kCsF * kCsFS];
  const int nstrip = (g.n1 + 3) / 4, nchunk = (L + kCsChunk - 1) / kCsChunk;
  const int nblk = nchunk * g.n1 * nstrip, per = (nblk + 7) / 8;
  const int q = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (q >= nblk) return;
  const int ch = q / (g.n1 * nstrip), rem = q % (g.n1 * nstrip);
  const int pa = rem / nstrip, b0 = (rem % nstrip) * 4;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int pb = b0 + w;
  const bool pv = pb < g.n1;
  const int i = pa * g.n1 + (pv ? pb : 0);
  // A[m][kk] = conj(U[k = m][pixel 4 s + kk]): lane supplies m = lane % 16, kk = lane / 16
  float ur[16], ui[16];
  {
    const int k = lane % 16;
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const cf x = pv && k < rcap ? U[((size_t)i * rcap + k) * 64 + st * 4 + lane / 16] : cf{0.f, 0.f};
      ur[st] = x.x;
      ui[st] = x.y;
    }
  }
  float fo[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = 4 * (lane / 16) + e;
    fo[e] = pv && k < rcap ? fk[(size_t)i * rcap + k] : 0.f;
  }
  const size_t NN = (size_t)g.N * g.N;
  const int x0 = 4 * b0, y0 = 4 * pa;
  const int lc0 = ch * kCsChunk, lc1 = min(L, lc0 + kCsChunk);
  cf nxt[kCsPer];
  auto load = [&](int l0) {
#pragma unroll
    for (int j = 0; j < kCsPer; ++j) {
      const int e = tid + 256 * j, f = e / (8 * kCsW), r2 = e % (8 * kCsW), y = r2 / kCsW, x = r2 % kCsW;
      nxt[j] = l0 + f < lc1 && x0 + x < g.N ? X[(size_t)(l0 + f) * NN + (size_t)(y0 + y) * g.N + x0 + x]
                                             : cf{0.f, 0.f};
    }
  };
  load(lc0);
  for (int l0 = lc0; l0 < lc1; l0 += kCsF) {
#pragma unroll
    for (int j = 0; j < kCsPer; ++j) {
      const int e = tid + 256 * j, f = e / (8 * kCsW), r2 = e % (8 * kCsW);
      S[f * kCsFS + r2] = nxt[j];
    }
    lds_sync();
    if (l0 + kCsF < lc1) load(l0 + kCsF);
    if (pv) {
      // four accumulation chains (Re, Im x even, odd pixel steps) keep the MFMA pipe busy
      f32x4 dr[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}}, di[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
      const cf* Sb = S + (lane % 16) * kCsFS + 4 * w;
#pragma unroll
      for (int st = 0; st < 16; ++st) {
        const int a = 4 * st + lane / 16, h = st & 1;
        const cf bv = Sb[(a >> 3) * kCsW + (a & 7)];
        dr[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(ur[st], bv.x, dr[h], 0, 0, 0);
        di[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(ur[st], bv.y, di[h], 0, 0, 0);
        dr[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(ui[st], bv.y, dr[h], 0, 0, 0);
        di[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ui[st], bv.x, di[h], 0, 0, 0);
      }
      const int f = l0 + lane % 16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * (lane / 16) + e;
        if (k < rcap && f < lc1)
          C[((size_t)i * rcap + k) * L + f] = cf{(dr[0][e] + dr[1][e]) * fo[e], (di[0][e] + di[1][e]) * fo[e]};
      }
    }
    lds_sync();
  }
}
inline int coef_strip_blocks(const PatchGeom& g, int L) {
  const int nblk = ((L + kCsChunk - 1) / kCsChunk) * g.n1 * ((g.n1 + 3) / 4);
  return 8 * ((nblk + 7) / 8);
}

__global__ __launch_bounds__(256) void k_coef_any(const cf* __restrict__ X, const cf* __restrict__ U,
                                                  const float* __restrict__ fk, PatchGeom g, int L, int rcap,
                                                  cf* __restrict__ C) {
  __shared__ cf Us[kMaxRllr][kMaxPP];
  __shared__ float fs[kMaxRllr];
  const int i = patch_of_block(g.Np);
  if (i < 0) return;
  const int PP = g.p * g.p;
  for (int idx = threadIdx.x; idx < rcap * PP; idx += 256) {
    const int k = idx / PP, a = idx % PP;
    Us[k][a] = U[((size_t)i * rcap + k) * PP + a];
  }
  if ((int)threadIdx.x < rcap) fs[threadIdx.x] = fk[(size_t)i * rcap + threadIdx.x];
  __syncthreads();
  const int oy = (i / g.n1) * g.s, ox = (i % g.n1) * g.s;
  const size_t NN = (size_t)g.N * g.N;
  for (int l = threadIdx.x; l < L; l += 256) {
    cf acc[kMaxRllr];
#pragma unroll
    for (int k = 0; k < kMaxRllr; ++k) acc[k] = cf{0.f, 0.f};
    const cf* Xl = X + (size_t)l * NN;
    for (int a = 0; a < PP; ++a) {
      const cf x = Xl[(size_t)(oy + a / g.p) * g.N + ox + a % g.p];
#pragma unroll
      for (int k = 0; k < kMaxRllr; ++k)
        if (k < rcap) acc[k] = cadd(acc[k], cconjmul(Us[k][a], x));
    }
#pragma unroll
    for (int k = 0; k < kMaxRllr; ++k)
      if (k < rcap) C[((size_t)i * rcap + k) * L + l] = cscale(acc[k], fs[k]);
  }
}

// X+[l][v] = (Z[l][v] + kappa sum_{i covers v} sum_k U[i][k][a_i(v)] C[i][k][l]) / (1 + kappa c(v))
// Block: 16 x 16 pixel tile (thread = pixel) and a range of frames; the C rows of the patches
// that cover the tile are staged in LDS for FCH frames at a time.
constexpr int kTile = 16;
constexpr int kXuFch = 8;

// The same X update when every pixel has at most 4 covering patches (p <= 2 s) and rcap <= RC:
// each thread keeps U[i][k][a_i(v)] of its covering patches in registers for the whole frame
// range, and the covering patches' C rows are staged in LDS 16 frames at a time.
constexpr int kXrFch = 16;
constexpr int kXrPad = 2;   // complex values of padding per patch block of Cs: its rows start on different banks
template <int RC, bool WITHZ>
__global__ __launch_bounds__(256) void k_xupdate_reg(const cf* __restrict__ Z, const cf* __restrict__ U,
                                                     const cf* __restrict__ C, PatchGeom g, int L, int rcap,
                                                     const double* __restrict__ kap_ptr, double kap_scale, int fpb,
                                                     cf* __restrict__ Xout) {
  extern __shared__ cf Cs[];   // [npt][rcap * kXrFch + kXrPad]
  const int ntx = g.N / kTile;
  const int ty = blockIdx.x / ntx, tx = blockIdx.x % ntx;
  const int t = threadIdx.x;
  const int py = ty * kTile + t / kTile, px = tx * kTile + t % kTile;
  const int v = py * g.N + px;
  const int cy0 = ty * kTile / g.s, cy1 = (ty * kTile + kTile - 1) / g.s;
  const int cx0 = tx * kTile / g.s, cx1 = (tx * kTile + kTile - 1) / g.s;
  const int alo = max(0, cy0 - g.ppc + 1), ahi = min(g.n1 - 1, cy1);
  const int blo = max(0, cx0 - g.ppc + 1), bhi = min(g.n1 - 1, cx1);
  const int nb = bhi - blo + 1, npt = (ahi - alo + 1) * nb;
  int a0, a1, b0, b1;
  cover_range(g, py / g.s, a0, a1);
  cover_range(g, px / g.s, b0, b1);
  const int na = a1 - a0 + 1, nbb = b1 - b0 + 1, ncov = na * nbb;
  const int PP = g.p * g.p;
  cf u[4][RC];
  int qo[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int a = a0 + (c < ncov ? c / nbb : 0), b = b0 + (c < ncov ? c % nbb : 0);
    const int i = a * g.n1 + b;
    qo[c] = ((a - alo) * nb + (b - blo)) * (rcap * kXrFch + kXrPad);
    const int ap = (py - a * g.s) * g.p + (px - b * g.s);
#pragma unroll
    for (int k = 0; k < RC; ++k)
      u[c][k] = (c < ncov && k < rcap) ? U[((size_t)i * rcap + k) * PP + ap] : cf{0.f, 0.f};
  }
  const float kap = WITHZ ? (float)(kap_ptr[0] * kap_scale) : 1.f;
  const float den = WITHZ ? 1.f / (1.f + kap * ncov) : 1.f;
  const int l0 = blockIdx.y * fpb, l1 = min(L, l0 + fpb);
  for (int lc = l0; lc < l1; lc += kXrFch) {
    const int nf = min(kXrFch, l1 - lc);
    __syncthreads();
    for (int idx = t; idx < npt * rcap * kXrFch; idx += 256) {
      const int f = idx % kXrFch, k = (idx / kXrFch) % rcap, q = idx / (kXrFch * rcap);
      const int i = (alo + q / nb) * g.n1 + blo + q % nb;
      Cs[q * (rcap * kXrFch + kXrPad) + k * kXrFch + f] = f < nf ? C[((size_t)i * rcap + k) * L + lc + f] : cf{0.f, 0.f};
    }
    __syncthreads();
    cf acc[kXrFch];
#pragma unroll
    for (int f = 0; f < kXrFch; ++f) acc[f] = cf{0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c < ncov) {
#pragma unroll
        for (int k = 0; k < RC; ++k) {
          if (k < rcap) {
            const float4* cs = (const float4*)(Cs + qo[c] + k * kXrFch);
#pragma unroll
            for (int f2 = 0; f2 < kXrFch / 2; ++f2) {
              const float4 w = cs[f2];
              acc[2 * f2] = cadd(acc[2 * f2], cmul(u[c][k], cf{w.x, w.y}));
              acc[2 * f2 + 1] = cadd(acc[2 * f2 + 1], cmul(u[c][k], cf{w.z, w.w}));
            }
          }
        }
      }
    }
#pragma unroll
    for (int f = 0; f < kXrFch; ++f)
      if (f < nf) {
        const size_t o = (size_t)(lc + f) * g.N * g.N + v;
        if (WITHZ) {
          const cf zv = Z[o];
          Xout[o] = cf{(zv.x + kap * acc[f].x) * den, (zv.y + kap * acc[f].y) * den};
        } else {
          Xout[o] = acc[f];
        }
      }
  }
}

// The same update on MFMA for 8 x 8 patches at stride 4. The 16 pixels of a 4 x 4 cell share
// their (up to) 4 covering patches, so a cell's frames are one complex product
//   X_cell[px][f] = sum_{k < rcap} sum_{c < 4} U_{i_c}[k][a_c(px)] C_{i_c}[k][f],
// a 16 x (4 rcap) by (4 rcap) x F matrix product. One wave per cell and 16-frame tile: the
// K-step k takes component k of the 4 patches (lane l: patch c = l / 16), so the A operands
// (U, kept in registers for all frames) and B operands (C, 16 consecutive frames per patch row)
// are plain loads; Re and Im come from four real 16x16x4 products. A block = 4 cells of one cell
// row and a range of frames; the 4 waves' tiles meet in LDS and leave as 128-byte rows. Blocks
// are dealt to the 8 XCDs (XCD = block mod 8) so that each XCD takes a band of rows_per cell rows
// for one frame chunk after another: cells of neighbouring rows and quads, which share covering
// patches, then read those patches' C through the same L2.
// ZB: Z is not read but formed here, Z = beta conj(V)^T (eq. (17)'s expansion; r <= 16) as four
// more K-steps of the same tile: A[pixel][kq] = beta[v][4 s + kq] (registers, all frames),
// B[kq][frame] = conj(V[frame][4 s + kq]); Re = br vr + bi vi, Im = bi vr - br vi.
template <int RC, bool WITHZ, bool ZB>
__global__ __launch_bounds__(256) void k_xupdate_mfma(const cf* __restrict__ Z, const cf* __restrict__ U,
                                                      const cf* __restrict__ C, const cf* __restrict__ beta,
                                                      const cf* __restrict__ Vb, int r, PatchGeom g, int L, int rcap,
                                                      const double* __restrict__ kap_ptr, double kap_scale, int fpb,
                                                      int rows_per, cf* __restrict__ Xout) {
  __shared__ cf T[16][4][16];
  const int nq = g.nc / 4;
  const int w = threadIdx.x >> 6;
  const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3, per = rows_per * nq;
  const int chunk = q / per, within = q % per;
  const int cy = xcd * rows_per + within / nq, cxb = (within % nq) * 4, cx = cxb + w;
  if (cy >= g.nc) return;   // the whole block: no barrier has been reached
  const int lane = threadIdx.x & 63, c = lane >> 4, px = lane & 15;
  const int a = cy - 1 + (c >> 1), b = cx - 1 + (c & 1);   // covering patch c of this cell
  const bool pv = a >= 0 && a < g.n1 && b >= 0 && b < g.n1;
  const int i = pv ? a * g.n1 + b : 0;
  const int ap = (4 * (cy - a) + (px >> 2)) * 8 + 4 * (cx - b) + (px & 3);   // pixel px inside patch c
  float ur[RC], ui[RC], un[RC];
#pragma unroll
  for (int k = 0; k < RC; ++k) {
    const cf x = pv && k < rcap ? U[((size_t)i * rcap + k) * 64 + ap] : cf{0.f, 0.f};
    ur[k] = x.x;
    ui[k] = x.y;
    un[k] = -x.y;
  }
  const float kap = WITHZ ? (float)(kap_ptr[0] * kap_scale) : 1.f;
  // 1 / (1 + kap c(v)) of each of the block's 4 cells: a thread stores pixels of all four, and
  // c(v) (the patches covering the cell) is smaller at the image's left and right edges
  float den[4];
#pragma unroll
  for (int qc = 0; qc < 4; ++qc) {
    int ncov = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int qa = cy - 1 + (q >> 1), qb = cxb + qc - 1 + (q & 1);
      ncov += qa >= 0 && qa < g.n1 && qb >= 0 && qb < g.n1;
    }
    den[qc] = WITHZ ? 1.f / (1.f + kap * ncov) : 1.f;
  }
  const int l0 = chunk * fpb, l1 = min(L, l0 + fpb);
  const cf* Ci = C + (size_t)i * rcap * L;
  const size_t NN = (size_t)g.N * g.N;
  float zbr[4], zbi[4], zbn[4];
  const int nzs = (r + 3) / 4;
  if constexpr (ZB) {
    const size_t vpx = (size_t)(4 * cy + (px >> 2)) * g.N + 4 * cx + (px & 3);   // pixel px of this cell
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * st + c;
      const cf bb = k < r ? beta[vpx * r + k] : cf{0.f, 0.f};
      zbr[st] = bb.x;
      zbi[st] = bb.y;
      zbn[st] = -bb.x;
    }
  }
  for (int f0 = l0; f0 < l1; f0 += 16) {
    const int f = f0 + px;
    const bool fv = pv && f < l1;
    cf bv[RC];
#pragma unroll
    for (int k = 0; k < RC; ++k) bv[k] = fv && k < rcap ? Ci[(size_t)k * L + f] : cf{0.f, 0.f};
    f32x4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < RC; ++k) {
      if (k < rcap) {   // uniform
        accr = __builtin_amdgcn_mfma_f32_16x16x4f32(ur[k], bv[k].x, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x4f32(ur[k], bv[k].y, acci, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x4f32(un[k], bv[k].y, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x4f32(ui[k], bv[k].x, acci, 0, 0, 0);
      }
    }
    f32x4 zr = {0.f, 0.f, 0.f, 0.f}, zi = {0.f, 0.f, 0.f, 0.f};
    if constexpr (ZB) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (st < nzs) {   // uniform
          const int k = 4 * st + c;
          const cf vv = f < l1 && k < r ? Vb[(size_t)f * r + k] : cf{0.f, 0.f};
          zr = __builtin_amdgcn_mfma_f32_16x16x4f32(zbr[st], vv.x, zr, 0, 0, 0);
          zr = __builtin_amdgcn_mfma_f32_16x16x4f32(zbi[st], vv.y, zr, 0, 0, 0);
          zi = __builtin_amdgcn_mfma_f32_16x16x4f32(zbi[st], vv.x, zi, 0, 0, 0);
          zi = __builtin_amdgcn_mfma_f32_16x16x4f32(zbn[st], vv.y, zi, 0, 0, 0);
        }
      }
    }
    // accumulator element e: cell pixel 4 (lane / 16) + e (row lane / 16, column e), frame
    // f0 + lane % 16; staged as T[frame][cell row][16 pixels of the 4 cells] so that the block
    // reads Z and writes X in 128-byte rows (ZB: the finished X of this wave's cell)
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (ZB)
        T[px][c][4 * w + e] = cf{(zr[e] + kap * accr[e]) * den[w], (zi[e] + kap * acci[e]) * den[w]};
      else
        T[px][c][4 * w + e] = cf{accr[e], acci[e]};
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int fr = (threadIdx.x >> 6) + 4 * q, row = (threadIdx.x >> 4) & 3, x16 = threadIdx.x & 15;
      if (f0 + fr < l1) {
        const size_t o = (size_t)(f0 + fr) * NN + (size_t)(4 * cy + row) * g.N + 4 * cxb + x16;
        const cf acc = T[fr][row][x16];
        if (WITHZ && !ZB) {
          const cf zv = Z[o];
          const float dn = den[x16 >> 2];   // the cell of this column
          Xout[o] = cf{(zv.x + kap * acc.x) * dn, (zv.y + kap * acc.y) * dn};
        } else {
          Xout[o] = acc;
        }
      }
    }
  }
}

template <bool WITHZ>
__global__ __launch_bounds__(256) void k_xupdate(const cf* __restrict__ Z, const cf* __restrict__ U,
                                                 const cf* __restrict__ C, PatchGeom g, int L, int rcap,
                                                 const double* __restrict__ kap_ptr, double kap_scale, int fpb,
                                                 cf* __restrict__ Xout) {
  extern __shared__ cf Cs[];   // [npt][rcap][kXuFch]
  const int ntx = g.N / kTile;
  const int ty = blockIdx.x / ntx, tx = blockIdx.x % ntx;
  const int t = threadIdx.x;
  const int py = ty * kTile + t / kTile, px = tx * kTile + t % kTile;
  const int v = py * g.N + px;
  const int cy0 = ty * kTile / g.s, cy1 = (ty * kTile + kTile - 1) / g.s;
  const int cx0 = tx * kTile / g.s, cx1 = (tx * kTile + kTile - 1) / g.s;
  const int alo = max(0, cy0 - g.ppc + 1), ahi = min(g.n1 - 1, cy1);
  const int blo = max(0, cx0 - g.ppc + 1), bhi = min(g.n1 - 1, cx1);
  const int na = ahi - alo + 1, nb = bhi - blo + 1, npt = na * nb;
  // this pixel's covering patches and in-patch offsets
  int a0, a1, b0, b1;
  cover_range(g, py / g.s, a0, a1);
  cover_range(g, px / g.s, b0, b1);
  const int cov = (a1 - a0 + 1) * (b1 - b0 + 1);
  const float kap = WITHZ ? (float)(kap_ptr[0] * kap_scale) : 1.f;
  const float den = WITHZ ? 1.f / (1.f + kap * cov) : 1.f;
  const int l0 = blockIdx.y * fpb, l1 = min(L, l0 + fpb);
  for (int lc = l0; lc < l1; lc += kXuFch) {
    const int nf = min(kXuFch, l1 - lc);
    __syncthreads();
    for (int idx = t; idx < npt * rcap * kXuFch; idx += 256) {
      const int f = idx % kXuFch, k = (idx / kXuFch) % rcap, q = idx / (kXuFch * rcap);
      const int i = (alo + q / nb) * g.n1 + blo + q % nb;
      Cs[idx] = f < nf ? C[((size_t)i * rcap + k) * L + lc + f] : cf{0.f, 0.f};
    }
    __syncthreads();
    cf acc[kXuFch];
#pragma unroll
    for (int f = 0; f < kXuFch; ++f) acc[f] = cf{0.f, 0.f};
    for (int a = a0; a <= a1; ++a)
      for (int b = b0; b <= b1; ++b) {
        const int i = a * g.n1 + b;
        const int q = (a - alo) * nb + (b - blo);
        const int ap = (py - a * g.s) * g.p + (px - b * g.s);
        for (int k = 0; k < rcap; ++k) {
          const cf u = U[((size_t)i * rcap + k) * g.p * g.p + ap];
          const cf* cs = Cs + ((size_t)q * rcap + k) * kXuFch;
#pragma unroll
          for (int f = 0; f < kXuFch; ++f) acc[f] = cadd(acc[f], cmul(u, cs[f]));
        }
      }
#pragma unroll
    for (int f = 0; f < kXuFch; ++f)
      if (f < nf) {
        const size_t o = (size_t)(lc + f) * g.N * g.N + v;
        if (WITHZ) {
          const cf zv = Z[o];
          Xout[o] = cf{(zv.x + kap * acc[f].x) * den, (zv.y + kap * acc[f].y) * den};
        } else {
          Xout[o] = acc[f];   // Q*(U_r C) alone
        }
      }
  }
}

__global__ __launch_bounds__(256) void k_sum_d(const double* __restrict__ a, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += a[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ------------------------------------------------------------------ workspace layout
struct LlrWs {
  cf* G;        // [Np][PP][PP]
  double* dd;   // [Np][PP]
  double* ee;   // [Np][PP]
  dcplx* refl;  // [Np][PP][PP]
  double* rtau; // [Np][PP]
  dcplx* ph;    // [Np][PP]
  double* nuc;  // [Np]
  double* z;    // [Np][rcap][PP]
  double* lam;  // [Np][rcap]
  size_t bytes;
};

static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

LlrWs llr_ws_layout(const PatchGeom& g, int rcap, void* base) {
  const size_t PP = (size_t)g.p * g.p, Np = g.Np;
  LlrWs w{};
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = p ? p + off : nullptr;
    off += al(b);
    return q;
  };
  w.G = (cf*)take(std::max(Np * PP * PP, (size_t)g.nc * g.nc * 5 * 256) * sizeof(cf));   // dense or cell-pair Grams
  w.dd = (double*)take(Np * PP * 8);
  w.ee = (double*)take(Np * PP * 8);
  w.refl = (dcplx*)take(Np * PP * PP * sizeof(dcplx));
  w.rtau = (double*)take(Np * PP * 8);
  w.ph = (dcplx*)take(Np * PP * sizeof(dcplx));
  w.nuc = (double*)take(Np * 8);
  w.z = (double*)take(Np * rcap * PP * 8);
  w.lam = (double*)take(Np * rcap * 8);
  w.bytes = off;
  return w;
}

// Eigen-analysis of every patch of X: U [Np][rcap][PP] (FP32), f [Np][rcap], nuc_out (device
// double) = sum of all singular values.
mrf_status llr_analyse(const cf* X, const PatchGeom& g, int L, double tau, int rcap, void* ws, cf* U, float* f,
                       double* nuc_out, double* lam_out, hipStream_t s) {
  const int PP = g.p * g.p;
  LlrWs w = llr_ws_layout(g, rcap, ws);
  const int nb = patch_blocks(g.Np);
  const bool cells = gram_cells_ok(g);
  if (cells)
    MRF_LAUNCH("llr_gram", s, k_gram_cells<<<gram_cells_blocks(g), 64 * kGcW, 0, s>>>(X, g.N, g.nc, L, w.G));
  else if (PP == 64) MRF_LAUNCH("llr_gram", s, k_gram<64><<<nb, GramCfg<64>::NTHR, 0, s>>>(X, g, L, w.G));
  else if (PP == 16) MRF_LAUNCH("llr_gram", s, k_gram<16><<<nb, GramCfg<16>::NTHR, 0, s>>>(X, g, L, w.G));
  else if (PP == 32 || PP == 48) return fail(MRF_SHAPE, "llr: p^2 must be 16 or 64 (or < 16)");
  else if (PP < 16) MRF_LAUNCH("llr_gram", s, k_gram_small<<<nb, 256, 0, s>>>(X, g, L, w.G));
  else return fail(MRF_SHAPE, "llr: p^2 must be 16 or 64 (or < 16)");
  MRF_LAUNCH("llr_tridiag", s,
             k_tridiag<<<nb, 64 * kTdW, 0, s>>>(cells ? nullptr : w.G, cells ? w.G : nullptr, g, g.Np, PP, w.dd, w.ee, w.refl,
                                          w.rtau, w.ph));
  MRF_LAUNCH("llr_eig", s, k_eig_val<<<nb, 64, 0, s>>>(w.dd, w.ee, g.Np, PP, tau, rcap, w.nuc, w.lam, f, lam_out));
  const int nv64 = (int)ceil_div((long)g.Np * rcap, 64L);
  if (PP == 64)
    MRF_LAUNCH("llr_eigvec", s, k_eig_vec_reg<64><<<nv64, 64, 0, s>>>(w.dd, w.ee, w.lam, f, g.Np, rcap, w.z));
  else if (PP == 16)
    MRF_LAUNCH("llr_eigvec", s, k_eig_vec_reg<16><<<nv64, 64, 0, s>>>(w.dd, w.ee, w.lam, f, g.Np, rcap, w.z));
  else
    MRF_LAUNCH("llr_eigvec", s,
               k_eig_vec<<<(int)ceil_div((long)g.Np * rcap, (long)kEvT), kEvT, 0, s>>>(w.dd, w.ee, w.lam, f, g.Np, PP,
                                                                                     rcap, w.z));
  const int nbw = std::max(1, (std::min(rcap, PP) + 3) / 4);   // waves: four vectors each
  MRF_LAUNCH("llr_backxf", s, k_backxf<<<nb, 64 * nbw, 0, s>>>(w.z, w.lam, w.refl, w.rtau, w.ph, g.Np, PP, rcap, U));
  MRF_LAUNCH("llr_nuc_sum", s, k_sum_d<<<1, 256, 0, s>>>(w.nuc, g.Np, nuc_out));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status llr_coef(const cf* X, const PatchGeom& g, int L, int rcap, const cf* U, const float* f, cf* C,
                    hipStream_t s) {
  const int PP = g.p * g.p, nb = patch_blocks(g.Np);
  if (g.p == 8 && g.s == 4 && rcap <= 16)
    MRF_LAUNCH("llr_coef", s, k_coef_strip<<<coef_strip_blocks(g, L), 256, 0, s>>>(X, U, f, g, L, rcap, C));
  else if (PP == 64) MRF_LAUNCH("llr_coef", s, k_coef<64><<<nb, 256, 0, s>>>(X, U, f, g, L, rcap, C));
  else if (PP == 16) MRF_LAUNCH("llr_coef", s, k_coef<16><<<nb, 256, 0, s>>>(X, U, f, g, L, rcap, C));
  else MRF_LAUNCH("llr_coef", s, k_coef_any<<<nb, 256, 0, s>>>(X, U, f, g, L, rcap, C));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// The X update with Z = beta conj(V)^T formed inside the kernel instead of read (the expansion of
// eq. (17) fused into eq. (23)): for 8 x 8 patches at stride 4 with rcap, r <= 16.
bool llr_xupdate_beta_ok(const PatchGeom& g, int rcap, int r) {
  return g.p == 8 && g.s == 4 && g.N % kTile == 0 && rcap <= 16 && r >= 1 && r <= 16;
}
mrf_status llr_xupdate_beta(const cf* beta, const cf* V, int r, const cf* U, const cf* C, const PatchGeom& g, int L,
                            int rcap, const double* kap_dev, double kap_scale, cf* Xout, hipStream_t s) {
  if (!llr_xupdate_beta_ok(g, rcap, r)) return fail(MRF_NOT_SUPPORTED, "x update from beta: geometry not supported");
#ifndef MRF_XU_FPB
#define MRF_XU_FPB 256
#endif
  const int fpb = MRF_XU_FPB;
  const int rows_per = (g.nc + 7) / 8;
  const int grid = 8 * rows_per * (g.nc / 4) * ((L + fpb - 1) / fpb);
  if (rcap <= 10)
    MRF_LAUNCH("llr_xupdate", s, k_xupdate_mfma<10, true, true><<<grid, 256, 0, s>>>(nullptr, U, C, beta, V, r, g, L, rcap,
                                                                                   kap_dev, kap_scale, fpb, rows_per,
                                                                                   Xout));
  else
    MRF_LAUNCH("llr_xupdate", s, k_xupdate_mfma<16, true, true><<<grid, 256, 0, s>>>(nullptr, U, C, beta, V, r, g, L, rcap,
                                                                                   kap_dev, kap_scale, fpb, rows_per,
                                                                                   Xout));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status llr_xupdate(const cf* Z, const cf* U, const cf* C, const PatchGeom& g, int L, int rcap,
                       const double* kap_dev, double kap_scale, cf* Xout, hipStream_t s) {
  if (g.N % kTile != 0) return fail(MRF_SHAPE, "x update: N must be a multiple of 16");
  const int ntile = (g.N / kTile) * (g.N / kTile);
  const int ca = kTile / g.s + g.ppc;   // covering patches per tile side (upper bound)
  if (g.p == 8 && g.s == 4 && rcap <= 16) {
    const int fpb = 64;
    const int rows_per = (g.nc + 7) / 8;   // cell rows per XCD band
    const int grid = 8 * rows_per * (g.nc / 4) * ((L + fpb - 1) / fpb);
#define MRF_XM(RCv, W, NAME, ZP, KP, KS)                                                                  \
  MRF_LAUNCH(NAME, s, k_xupdate_mfma<RCv, W, false><<<grid, 256, 0, s>>>(ZP, U, C, nullptr, nullptr, 0, g, L, rcap, KP, \
                                                                         KS, fpb, rows_per, Xout))
    if (rcap <= 10) {
      if (Z) MRF_XM(10, true, "llr_xupdate", Z, kap_dev, kap_scale);
      else MRF_XM(10, false, "llr_qtp", nullptr, nullptr, 1.0);
    } else {
      if (Z) MRF_XM(16, true, "llr_xupdate", Z, kap_dev, kap_scale);
      else MRF_XM(16, false, "llr_qtp", nullptr, nullptr, 1.0);
    }
#undef MRF_XM
    MRF_CHECK_LAUNCH();
    return MRF_OK;
  }
  if (g.ppc <= 2 && rcap <= 16) {
    const size_t lds = (size_t)ca * ca * (rcap * kXrFch + kXrPad) * sizeof(cf);
    if (lds <= 64 * 1024) {
      // frame groups: enough blocks to fill the chip, whole 16-frame chunks
      const int fpb = std::max(kXrFch, ((L + 15) / 16 + kXrFch - 1) / kXrFch * kXrFch);
      dim3 grid(ntile, (L + fpb - 1) / fpb);
#define MRF_XR(RCv, W, NAME, ZP, KP, KS)                                                                  \
  MRF_LAUNCH(NAME, s, k_xupdate_reg<RCv, W><<<grid, 256, lds, s>>>(ZP, U, C, g, L, rcap, KP, KS, fpb, Xout))
      if (rcap <= 10) {
        if (Z) MRF_XR(10, true, "llr_xupdate", Z, kap_dev, kap_scale);
        else MRF_XR(10, false, "llr_qtp", nullptr, nullptr, 1.0);
      } else {
        if (Z) MRF_XR(16, true, "llr_xupdate", Z, kap_dev, kap_scale);
        else MRF_XR(16, false, "llr_qtp", nullptr, nullptr, 1.0);
      }
#undef MRF_XR
      MRF_CHECK_LAUNCH();
      return MRF_OK;
    }
  }
  const size_t lds = (size_t)ca * ca * rcap * kXuFch * sizeof(cf);
  if (lds > 64 * 1024) return fail(MRF_SHAPE, "x update: too many patches per tile");
  const int fpb = std::max(kXuFch, ((L + 63) / 64 + kXuFch - 1) / kXuFch * kXuFch);
  dim3 grid(ntile, (L + fpb - 1) / fpb);
  if (Z)
    MRF_LAUNCH("llr_xupdate", s,
               k_xupdate<true><<<grid, 256, lds, s>>>(Z, U, C, g, L, rcap, kap_dev, kap_scale, fpb, Xout));
  else
    MRF_LAUNCH("llr_qtp", s,
               k_xupdate<false><<<grid, 256, lds, s>>>(nullptr, U, C, g, L, rcap, nullptr, 1.0, fpb, Xout));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

size_t llr_ws_bytes(const PatchGeom& g, int rcap) { return llr_ws_layout(g, rcap, nullptr).bytes; }

__global__ void k_set_d(double* __restrict__ p, double v) { p[0] = v; }

}  // namespace mrf

using namespace mrf;

extern "C" mrf_status mrf_llr_workspace_size(int n, int L, int p, int s, int rank_cap, size_t* bytes) {
  clear_error();
  PatchGeom g;
  MRF_REQUIRE(bytes, MRF_INVALID_ARG, "llr_workspace_size: null output");
  MRF_REQUIRE(make_geom(n, p, s, &g), MRF_SHAPE, "llr_workspace_size: need p % s == 0 and (n - p) % s == 0");
  MRF_REQUIRE(rank_cap >= 1 && rank_cap <= kMaxRllr && L >= 1, MRF_INVALID_ARG, "llr_workspace_size: bad rank cap or L");
  const size_t PP = (size_t)p * p;
  *bytes = llr_ws_bytes(g, rank_cap) + al((size_t)g.Np * rank_cap * PP * sizeof(cf)) + al((size_t)g.Np * rank_cap * 4) +
           al((size_t)g.Np * rank_cap * L * sizeof(cf));
  return MRF_OK;
}

extern "C" mrf_status mrf_llr_prox(const mrf_c64* X, mrf_c64* QtP, int n, int L, int p, int s, float tau, int rank_cap,
                                   double* nuc_norm, void* ws, size_t ws_bytes, hipStream_t st) {
  clear_error();
  PatchGeom g;
  MRF_REQUIRE(X && QtP && nuc_norm, MRF_INVALID_ARG, "llr_prox: null argument");
  MRF_REQUIRE(make_geom(n, p, s, &g), MRF_SHAPE, "llr_prox: need p % s == 0 and (n - p) % s == 0");
  MRF_REQUIRE(p * p <= kMaxPP && (p * p == 64 || p * p == 16 || p * p < 16), MRF_SHAPE, "llr_prox: p must be 2, 3, 4 or 8");
  MRF_REQUIRE(n % 16 == 0, MRF_SHAPE, "llr_prox: n must be a multiple of 16");
  MRF_REQUIRE(rank_cap >= 1 && rank_cap <= kMaxRllr && L >= 1 && tau >= 0.f, MRF_INVALID_ARG, "llr_prox: bad rank cap, L or tau");
  size_t need = 0;
  mrf_llr_workspace_size(n, L, p, s, rank_cap, &need);
  MRF_REQUIRE(ws && ws_bytes >= need, MRF_WORKSPACE, "llr_prox: workspace too small");
  const size_t PP = (size_t)p * p;
  char* base = (char*)ws;
  size_t off = llr_ws_bytes(g, rank_cap);
  cf* U = (cf*)(base + off); off += al((size_t)g.Np * rank_cap * PP * sizeof(cf));
  float* f = (float*)(base + off); off += al((size_t)g.Np * rank_cap * 4);
  cf* C = (cf*)(base + off); off += al((size_t)g.Np * rank_cap * L * sizeof(cf));
  mrf_status r = llr_analyse((const cf*)X, g, L, tau, rank_cap, ws, U, f, nuc_norm, nullptr, st);
  if (r != MRF_OK) return r;
  r = llr_coef((const cf*)X, g, L, rank_cap, U, f, C, st);
  if (r != MRF_OK) return r;
  return llr_xupdate(nullptr, U, C, g, L, rank_cap, nullptr, 1.0, (cf*)QtP, st);
}

extern "C" mrf_status mrf_llr_xupdate_workspace_size(int n, int L, int p, int s, int rank_cap, size_t* bytes) {
  mrf_status e = mrf_llr_workspace_size(n, L, p, s, rank_cap, bytes);
  if (e == MRF_OK) *bytes += 256;   // the device copy of kappa
  return e;
}

extern "C" mrf_status mrf_llr_xupdate(const mrf_c64* X, const mrf_c64* Z, const mrf_c64* beta_coef, const mrf_c64* V,
                                      int r, int n, int L, int p, int s, float tau, int rank_cap, double kappa,
                                      mrf_c64* Xout, void* ws, size_t ws_bytes, hipStream_t st) {
  clear_error();
  PatchGeom g;
  MRF_REQUIRE(X && Xout, MRF_INVALID_ARG, "llr_xupdate: null argument");
  MRF_REQUIRE((Z != nullptr) != (beta_coef != nullptr), MRF_INVALID_ARG, "llr_xupdate: give exactly one of Z and beta_coef");
  MRF_REQUIRE(!beta_coef || (V && r >= 1 && r <= 16), MRF_INVALID_ARG, "llr_xupdate: beta_coef needs V and 1 <= r <= 16");
  MRF_REQUIRE(X != (const mrf_c64*)Xout && Z != (const mrf_c64*)Xout, MRF_INVALID_ARG,
              "llr_xupdate: Xout must not alias X or Z");
  MRF_REQUIRE(make_geom(n, p, s, &g), MRF_SHAPE, "llr_xupdate: need p % s == 0 and (n - p) % s == 0");
  MRF_REQUIRE(p * p <= kMaxPP && (p * p == 64 || p * p == 16 || p * p < 16), MRF_SHAPE, "llr_xupdate: p must be 2, 3, 4 or 8");
  MRF_REQUIRE(n % 16 == 0, MRF_SHAPE, "llr_xupdate: n must be a multiple of 16");
  MRF_REQUIRE(rank_cap >= 1 && rank_cap <= kMaxRllr && L >= 1 && tau >= 0.f && kappa >= 0.0 && std::isfinite(kappa),
              MRF_INVALID_ARG, "llr_xupdate: bad rank cap, L, tau or kappa");
  MRF_REQUIRE(!beta_coef || llr_xupdate_beta_ok(g, rank_cap, r), MRF_NOT_SUPPORTED,
              "llr_xupdate: Z from beta_coef needs 8 x 8 patches at stride 4");
  size_t need = 0;
  mrf_llr_xupdate_workspace_size(n, L, p, s, rank_cap, &need);
  MRF_REQUIRE(ws && ws_bytes >= need, MRF_WORKSPACE, "llr_xupdate: workspace too small");
  const size_t PP = (size_t)p * p;
  char* base = (char*)ws;
  size_t off = llr_ws_bytes(g, rank_cap);
  cf* U = (cf*)(base + off); off += al((size_t)g.Np * rank_cap * PP * sizeof(cf));
  float* f = (float*)(base + off); off += al((size_t)g.Np * rank_cap * 4);
  cf* C = (cf*)(base + off); off += al((size_t)g.Np * rank_cap * L * sizeof(cf));
  double* kap = (double*)(base + off);
  double* nuc = kap + 1;
  MRF_LAUNCH("llr_set_kappa", st, k_set_d<<<1, 1, 0, st>>>(kap, kappa));
  mrf_status e = llr_analyse((const cf*)X, g, L, tau, rank_cap, ws, U, f, nuc, nullptr, st);
  if (e != MRF_OK) return e;
  if ((e = llr_coef((const cf*)X, g, L, rank_cap, U, f, C, st))) return e;
  if (beta_coef)
    return llr_xupdate_beta((const cf*)beta_coef, (const cf*)V, r, U, C, g, L, rank_cap, kap, 1.0, (cf*)Xout, st);
  return llr_xupdate((const cf*)Z, U, C, g, L, rank_cap, kap, 1.0, (cf*)Xout, st);
}
