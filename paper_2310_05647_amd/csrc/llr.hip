// Locally low-rank proximal step (Sec. III-C, eqs. (20), (22), (23)).
//
// For every patch i the Casorati matrix P_i = Q_{q_i}(X) (p^2 x L) is thresholded:
//   P_i = U S V^H,  P'_i = U_r diag(max(sigma - tau, 0)) V_r^H  (at most r_cap values kept)
// computed without the L-sided vectors: with the Gram G_i = P_i P_i^H = U S^2 U^H,
//   P'_i = U_r diag(f) U_r^H P_i,   f_k = max(sigma_k - tau, 0) / sigma_k,   sigma_k = sqrt(lambda_k).
// Steps (kernels):
//   k_gram      G_i on MFMA (v_mfma_f32_16x16x4f32) from the real [Re P | Im P] blocks, FP32
//   k_tridiag   complex Householder reduction of G_i to a real symmetric tridiagonal T, in FP64
//   k_eig_tri   all eigenvalues of T by Sturm bisection (one lane per eigenvalue), the nuclear
//               norm sum_k sigma_k, and the top r_cap eigenvectors by inverse iteration
//   k_backxf    eigenvectors of G_i = Q D z (reflectors Q, phases D), stored with f_k
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

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
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

// G_i = P_i P_i^H, p^2 = PP. Re G = A1 A1^T, Im G = A2 A1^T with A1 = [Re P | Im P],
// A2 = [Im P | -Re P] over the interleaved K index k = 2 l + {0: re, 1: im}. Only the upper
// 16 x 16 tiles are computed; the kernel writes both triangles.
template <int PP>
__global__ __launch_bounds__(256) void k_gram(const cf* __restrict__ X, PatchGeom g, int L, cf* __restrict__ G) {
  constexpr int NT = PP / 16;                   // tiles per side
  constexpr int NUP = NT * (NT + 1) / 2;        // upper tiles
  constexpr int FCH = 64;                       // frames per LDS chunk
  constexpr int TPW = (2 * NUP + 3) / 4;        // accumulators per wave (re and im tiles)
  __shared__ cf P[FCH][PP];
  const int i = patch_of_block(g.Np);
  if (i < 0) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int oy = (i / g.n1) * g.s, ox = (i % g.n1) * g.s;
  const size_t NN = (size_t)g.N * g.N;
  f32x4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  // accumulator q of wave w is job j = w * TPW + q: tile (ta, tb) = upper[j % NUP], part = j / NUP
  for (int l0 = 0; l0 < L; l0 += FCH) {
    const int nf = min(FCH, L - l0);
    for (int idx = tid; idx < FCH * PP; idx += 256) {
      const int f = idx / PP, a = idx % PP;
      P[f][a] = f < nf ? X[(size_t)(l0 + f) * NN + (size_t)(oy + a / g.p) * g.N + ox + a % g.p] : cf{0.f, 0.f};
    }
    __syncthreads();
    for (int k0 = 0; k0 < 2 * FCH; k0 += 4) {
      const int k = k0 + lane / 16;
      const int f = k >> 1, part = k & 1;
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        const int j = w * TPW + q;
        if (j < 2 * NUP) {
          int u = j % NUP, ta = 0;
          while (u >= NT - ta) {
            u -= NT - ta;
            ++ta;
          }
          const int tb = ta + u;
          const cf pa = P[f][ta * 16 + lane % 16];
          const cf pb = P[f][tb * 16 + lane % 16];
          const float bval = part ? pb.y : pb.x;                  // A1[b][k]
          float aval;
          if (j < NUP) aval = part ? pa.y : pa.x;                 // A1[a][k]
          else aval = part ? -pa.x : pa.y;                        // A2[a][k]
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(aval, bval, acc[q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  cf* Gi = G + (size_t)i * PP * PP;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int j = w * TPW + q;
    if (j < 2 * NUP) {
      int u = j % NUP, ta = 0;
      while (u >= NT - ta) {
        u -= NT - ta;
        ++ta;
      }
      const int tb = ta + u;
      const bool im = j >= NUP;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int a = ta * 16 + 4 * (lane / 16) + e, b = tb * 16 + lane % 16;
        if (ta == tb && a > b) continue;   // diagonal tiles: the upper half writes both halves
        float* ga = (float*)&Gi[(size_t)a * PP + b];
        float* gb = (float*)&Gi[(size_t)b * PP + a];
        if (!im) {
          ga[0] = acc[q][e];
          gb[0] = acc[q][e];
        } else {
          const float vi = a == b ? 0.f : acc[q][e];
          ga[1] = vi;
          gb[1] = -vi;
        }
      }
    }
  }
}

// Small patches (p^2 < 16): plain FP32 accumulation, one thread per matrix entry.
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
// One wave per patch; A (n x n, Hermitian, FP64) in LDS, lane = row. For k = 0 .. n-3:
//   x = A[k+1:, k], alpha = ||x||, phase = x0/|x0|, beta = -phase alpha, v = x - beta e1,
//   tau = 1 / (alpha (alpha + |x0|)) so that H = I - tau v v^H maps x to beta e1;
//   p = tau A22 v, K = tau/2 v^H p, w = p - K v, A22 -= v w^H + w v^H.
// The reflectors are written out (v, tau); T has diagonal d and sub-diagonal e (complex), then
// the phases D make it real: D_0 = 1, D_{k+1} = D_k e_k / |e_k|, e_k -> |e_k|.
__global__ __launch_bounds__(64) void k_tridiag(const cf* __restrict__ G, int Np, int n, double* __restrict__ dd,
                                               double* __restrict__ ee, dcplx* __restrict__ refl,
                                               double* __restrict__ rtau, dcplx* __restrict__ phase) {
  __shared__ dcplx A[kMaxPP][kMaxPP + 1];
  __shared__ dcplx vs[kMaxPP];
  const int i = patch_of_block(Np);
  if (i < 0) return;
  const int r = threadIdx.x;
  const cf* Gi = G + (size_t)i * n * n;
  if (r < n)
    for (int c = 0; c < n; ++c) {
      const cf x = Gi[(size_t)r * n + c];
      A[r][c] = dcplx{x.x, x.y};
    }
  __syncthreads();
  dcplx* Ri = refl + (size_t)i * n * n;     // reflector k stored in row k (entries k+1 .. n-1)
  dcplx ecur{0.0, 0.0};
  for (int k = 0; k < n - 2; ++k) {
    const bool below = r > k && r < n;
    const dcplx x = below ? A[r][k] : dcplx{0.0, 0.0};
    const double alpha = sqrt(wave_sum(below ? x.x * x.x + x.y * x.y : 0.0));
    const dcplx x0 = A[k + 1][k];
    const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
    dcplx ph = ax0 > 0 ? dcplx{x0.x / ax0, x0.y / ax0} : dcplx{1.0, 0.0};
    double tau = 0.0;
    dcplx v{0.0, 0.0};
    dcplx beta{0.0, 0.0};
    if (alpha > 0.0) {
      beta = dscale(ph, -alpha);
      tau = 1.0 / (alpha * (alpha + ax0));
      if (below) v = (r == k + 1) ? dsub(x, beta) : x;
    }
    if (r < n) Ri[(size_t)k * n + r] = below ? v : dcplx{0.0, 0.0};
    if (r == 0) rtau[(size_t)i * n + k] = tau;
    if (r == k) ecur = alpha > 0.0 ? beta : x0;   // lane k keeps e_k
    if (tau != 0.0) {
      vs[r] = v;
      __syncthreads();
      // p = tau A22 v (row r of A22)
      dcplx p{0.0, 0.0};
      if (below)
        for (int c = k + 1; c < n; ++c) p = dadd(p, dmul(A[r][c], vs[c]));
      p = dscale(p, tau);
      // K = tau/2 v^H p
      const double kr = wave_sum(below ? v.x * p.x + v.y * p.y : 0.0);
      const double ki = wave_sum(below ? v.x * p.y - v.y * p.x : 0.0);
      const dcplx K = dscale(dcplx{kr, ki}, 0.5 * tau);
      const dcplx wv = dsub(p, dmul(K, v));
      __syncthreads();
      vs[r] = v;
      __shared__ dcplx ws[kMaxPP];
      ws[r] = wv;
      __syncthreads();
      if (below)
        for (int c = k + 1; c < n; ++c) {
          // A[r][c] -= v_r conj(w_c) + w_r conj(v_c)
          const dcplx t1 = dmul(v, dcplx{ws[c].x, -ws[c].y});
          const dcplx t2 = dmul(wv, dcplx{vs[c].x, -vs[c].y});
          A[r][c] = dsub(A[r][c], dadd(t1, t2));
        }
      __syncthreads();
    }
  }
  if (r == n - 2) ecur = A[n - 1][n - 2];
  __syncthreads();
  // diagonal and real sub-diagonal; phases
  if (r < n) dd[(size_t)i * n + r] = A[r][r].x;
  __shared__ dcplx es[kMaxPP];
  es[r] = ecur;
  __syncthreads();
  if (r == 0) {
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

// Number of eigenvalues of the symmetric tridiagonal (d, e) smaller than x (Sturm sequence).
__device__ inline int sturm_count(const double* d, const double* e, int n, double x) {
  int c = 0;
  double q = d[0] - x;
  if (q < 0) ++c;
  for (int k = 1; k < n; ++k) {
    const double qq = fabs(q) < 1e-300 ? (q < 0 ? -1e-300 : 1e-300) : q;
    q = d[k] - x - e[k - 1] * e[k - 1] / qq;
    if (q < 0) ++c;
  }
  return c;
}

// One wave per patch. Lane j finds eigenvalue j (ascending) by bisection on the Sturm count;
// the sum of sigma = sqrt(max(lambda, 0)) is the patch's nuclear norm. Lanes 0 .. rcap-1 then
// each compute the eigenvector of the j-th largest eigenvalue by inverse iteration on T
// (tridiagonal LU with partial pivoting), re-orthogonalised inside clusters.
__global__ __launch_bounds__(64) void k_eig_tri(const double* __restrict__ dd, const double* __restrict__ ee, int Np,
                                               int n, double tau_thr, int rcap, double* __restrict__ nuc,
                                               double* __restrict__ zvec, float* __restrict__ fk,
                                               double* __restrict__ lam_out) {
  __shared__ double d[kMaxPP], e[kMaxPP], lam[kMaxPP];
  __shared__ double Z[kMaxRllr][kMaxPP];
  __shared__ double wrk[kMaxRllr][4][kMaxPP];
  const int i = patch_of_block(Np);
  if (i < 0) return;
  const int t = threadIdx.x;
  if (t < n) {
    d[t] = dd[(size_t)i * n + t];
    e[t] = ee[(size_t)i * n + t];
  }
  __syncthreads();
  // Gershgorin interval
  double lo = 0.0, hi = 0.0;
  for (int k = 0; k < n; ++k) {
    const double rad = (k > 0 ? e[k - 1] : 0.0) + (k < n - 1 ? e[k] : 0.0);
    lo = k == 0 ? d[k] - rad : fmin(lo, d[k] - rad);
    hi = k == 0 ? d[k] + rad : fmax(hi, d[k] + rad);
  }
  const double span = fmax(hi - lo, 1e-300);
  lo -= 1e-12 * span + 1e-300;
  hi += 1e-12 * span + 1e-300;
  double a = lo, b = hi;
  for (int it = 0; it < 80; ++it) {   // bisection: lambda_t (ascending) lies in (a, b]
    const double m = 0.5 * (a + b);
    if (m <= a || m >= b) break;
    if (t < n && sturm_count(d, e, n, m) > t) b = m;
    else a = m;
  }
  const double lt = 0.5 * (a + b);
  if (t < n) lam[t] = lt;
  const double sg = t < n ? sqrt(fmax(lt, 0.0)) : 0.0;
  const double tot = wave_sum(sg);
  if (t == 0) nuc[i] = tot;
  __syncthreads();
  // eigenvectors of the rcap largest eigenvalues
  const double scale = fmax(fabs(lo), fabs(hi));
  if (t < rcap && t < n) {
    const double lk = lam[n - 1 - t];
    const double sk = sqrt(fmax(lk, 0.0));
    const double f = sk > tau_thr ? (sk - tau_thr) / sk : 0.0;
    fk[(size_t)i * rcap + t] = (float)f;
    if (lam_out) lam_out[(size_t)i * rcap + t] = lk;
    double* y = Z[t];
    double* u0 = wrk[t][0];   // LU: U diagonal, first and second super-diagonals, multipliers
    double* u1 = wrk[t][1];
    double* u2 = wrk[t][2];
    double* ml = wrk[t][3];
    // LU with partial pivoting of (T - lk I); tiny pivots replaced by eps * scale
    const double eps = 1e-14 * scale + 1e-300;
    double dcur = d[0] - lk, ecur = n > 1 ? e[0] : 0.0;
    unsigned long long pivmask = 0ull;
    for (int k = 0; k < n - 1; ++k) {
      const double sub = e[k];
      double nd = d[k + 1] - lk, ne = k + 1 < n - 1 ? e[k + 1] : 0.0;
      if (fabs(dcur) >= fabs(sub)) {
        const double piv_v = fabs(dcur) < eps ? eps : dcur;
        u0[k] = piv_v; u1[k] = ecur; u2[k] = 0.0;
        ml[k] = sub / piv_v;
        dcur = nd - ml[k] * ecur;
        ecur = ne;
      } else {
        pivmask |= 1ull << k;
        u0[k] = sub; u1[k] = nd; u2[k] = ne;
        ml[k] = dcur / sub;
        dcur = ecur - ml[k] * nd;
        ecur = -ml[k] * ne;
      }
    }
    u0[n - 1] = fabs(dcur) < eps ? eps : dcur;
    for (int k = 0; k < n; ++k) y[k] = 1.0 + 0.01 * ((k * 37 + t * 11) % 7);
    for (int it = 0; it < 3; ++it) {
      // forward: apply the row interchanges and multipliers
      for (int k = 0; k < n - 1; ++k) {
        if ((pivmask >> k) & 1ull) {
          const double tmp = y[k];
          y[k] = y[k + 1];
          y[k + 1] = tmp - ml[k] * y[k];
        } else {
          y[k + 1] -= ml[k] * y[k];
        }
      }
      // back substitution with U (diagonal u0, super-diagonals u1, u2)
      for (int k = n - 1; k >= 0; --k) {
        double s = y[k];
        if (k + 1 < n) s -= u1[k] * y[k + 1];
        if (k + 2 < n) s -= u2[k] * y[k + 2];
        y[k] = s / u0[k];
      }
      double nr = 0.0;
      for (int k = 0; k < n; ++k) nr += y[k] * y[k];
      nr = 1.0 / sqrt(fmax(nr, 1e-300));
      for (int k = 0; k < n; ++k) y[k] *= nr;
    }
  }
  __syncthreads();
  // orthogonalise inside clusters (sequential over the vectors, in order)
  if (t == 0) {
    const int m = min(rcap, n);
    for (int k = 1; k < m; ++k) {
      for (int j = 0; j < k; ++j) {
        if (fabs(lam[n - 1 - k] - lam[n - 1 - j]) <= 1e-6 * scale) {
          double dot = 0.0;
          for (int q = 0; q < n; ++q) dot += Z[j][q] * Z[k][q];
          for (int q = 0; q < n; ++q) Z[k][q] -= dot * Z[j][q];
          double nr = 0.0;
          for (int q = 0; q < n; ++q) nr += Z[k][q] * Z[k][q];
          nr = 1.0 / sqrt(fmax(nr, 1e-300));
          for (int q = 0; q < n; ++q) Z[k][q] *= nr;
        }
      }
    }
  }
  __syncthreads();
  for (int k = 0; k < min(rcap, n); ++k)
    if (t < n) zvec[((size_t)i * rcap + k) * n + t] = Z[k][t];
}

// u_k = H_0 H_1 ... H_{n-3} D z_k for the rcap vectors; lane = row. Stores U[i][k][a] (FP32).
__global__ __launch_bounds__(64) void k_backxf(const double* __restrict__ zvec, const dcplx* __restrict__ refl,
                                              const double* __restrict__ rtau, const dcplx* __restrict__ phase,
                                              int Np, int n, int rcap, cf* __restrict__ U) {
  const int i = patch_of_block(Np);
  if (i < 0) return;
  const int r = threadIdx.x;
  const dcplx* Ri = refl + (size_t)i * n * n;
  for (int k = 0; k < rcap && k < n; ++k) {
    const double z = r < n ? zvec[((size_t)i * rcap + k) * n + r] : 0.0;
    dcplx u = r < n ? dscale(phase[(size_t)i * n + r], z) : dcplx{0.0, 0.0};
    for (int j = n - 3; j >= 0; --j) {
      const double tau = rtau[(size_t)i * n + j];
      if (tau == 0.0) continue;
      const dcplx v = r < n ? Ri[(size_t)j * n + r] : dcplx{0.0, 0.0};
      // u -= tau v (v^H u)
      const double dr = wave_sum(v.x * u.x + v.y * u.y);
      const double di = wave_sum(v.x * u.y - v.y * u.x);
      const dcplx c = dscale(dcplx{dr, di}, tau);
      u = dsub(u, dmul(v, c));
    }
    if (r < n) U[((size_t)i * rcap + k) * n + r] = cf{(float)u.x, (float)u.y};
  }
}

// C[i][k][l] = f_k sum_a conj(U[i][k][a]) X[l][pixel a of patch i]; block per patch, thread per frame.
__global__ __launch_bounds__(256) void k_coef(const cf* __restrict__ X, const cf* __restrict__ U,
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
  w.G = (cf*)take(Np * PP * PP * sizeof(cf));
  w.dd = (double*)take(Np * PP * 8);
  w.ee = (double*)take(Np * PP * 8);
  w.refl = (dcplx*)take(Np * PP * PP * sizeof(dcplx));
  w.rtau = (double*)take(Np * PP * 8);
  w.ph = (dcplx*)take(Np * PP * sizeof(dcplx));
  w.nuc = (double*)take(Np * 8);
  w.z = (double*)take(Np * rcap * PP * 8);
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
  if (PP == 64) MRF_LAUNCH("llr_gram", s, k_gram<64><<<nb, 256, 0, s>>>(X, g, L, w.G));
  else if (PP == 16) MRF_LAUNCH("llr_gram", s, k_gram<16><<<nb, 256, 0, s>>>(X, g, L, w.G));
  else if (PP == 32 || PP == 48) return fail(MRF_SHAPE, "llr: p^2 must be 16 or 64 (or < 16)");
  else if (PP < 16) MRF_LAUNCH("llr_gram", s, k_gram_small<<<nb, 256, 0, s>>>(X, g, L, w.G));
  else return fail(MRF_SHAPE, "llr: p^2 must be 16 or 64 (or < 16)");
  MRF_LAUNCH("llr_tridiag", s, k_tridiag<<<nb, 64, 0, s>>>(w.G, g.Np, PP, w.dd, w.ee, w.refl, w.rtau, w.ph));
  MRF_LAUNCH("llr_eig", s, k_eig_tri<<<nb, 64, 0, s>>>(w.dd, w.ee, g.Np, PP, tau, rcap, w.nuc, w.z, f, lam_out));
  MRF_LAUNCH("llr_backxf", s, k_backxf<<<nb, 64, 0, s>>>(w.z, w.refl, w.rtau, w.ph, g.Np, PP, rcap, U));
  MRF_LAUNCH("llr_nuc_sum", s, k_sum_d<<<1, 256, 0, s>>>(w.nuc, g.Np, nuc_out));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status llr_coef(const cf* X, const PatchGeom& g, int L, int rcap, const cf* U, const float* f, cf* C,
                    hipStream_t s) {
  MRF_LAUNCH("llr_coef", s, k_coef<<<patch_blocks(g.Np), 256, 0, s>>>(X, U, f, g, L, rcap, C));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status llr_xupdate(const cf* Z, const cf* U, const cf* C, const PatchGeom& g, int L, int rcap,
                       const double* kap_dev, double kap_scale, cf* Xout, hipStream_t s) {
  if (g.N % kTile != 0) return fail(MRF_SHAPE, "x update: N must be a multiple of 16");
  const int ntile = (g.N / kTile) * (g.N / kTile);
  const int ca = kTile / g.s + g.ppc;   // covering patches per tile side (upper bound)
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
