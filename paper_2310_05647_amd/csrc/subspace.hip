// Temporal subspace operators and dictionary matching (Sec. II-B eqs. (4)-(5); Sec. III-B eq. (17)).
//
//   P_S(X) = X V V^H, applied to every voxel's time course (eq. (17))
//   alpha = X V: per-voxel coefficients in the r-dimensional basis V [L][r]
//   Phi_D: k = argmax_m |<d_m, x>| / ||d_m||, eta = LUT[k], rho = max(Re<d_k, x> / ||d_k||^2, 0)
// The subspace match compares alpha with the projected atoms d_m V, normalised by the full-length
// norm ||d_m||; ties go to the lowest m. The match is a dense complex GEMM (voxels x atoms x r)
// run on MFMA (v_mfma_f32_16x16x4f32) with the arg-max fused into its epilogue.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.hpp"

#include "dict.hpp"

namespace mrf {

constexpr int kMaxR = 16;

// ---------------------------------------------------------------- dictionary preparation
// One block per atom: norm (double, fixed order) and projected unit atom (d_m V)/||d_m||.
__global__ __launch_bounds__(256) void k_dict_prep(const cf* __restrict__ atoms, const cf* __restrict__ V, int M,
                                                   int L, int r, float* __restrict__ norms, cf* __restrict__ dhr,
                                                   cf* __restrict__ dn) {
  __shared__ double red[256];
  __shared__ double accr[256][kMaxR];
  __shared__ double acci[256][kMaxR];
  const int m = blockIdx.x, t = threadIdx.x;
  const cf* d = atoms + (size_t)m * L;
  double s = 0.0;
  double ar[kMaxR], ai[kMaxR];
  for (int k = 0; k < kMaxR; ++k) ar[k] = ai[k] = 0.0;
  for (int l = t; l < L; l += 256) {
    const cf x = d[l];
    s += (double)x.x * x.x + (double)x.y * x.y;
    if (V)
      for (int k = 0; k < r; ++k) {
        const cf v = V[(size_t)l * r + k];
        ar[k] += (double)x.x * v.x - (double)x.y * v.y;
        ai[k] += (double)x.x * v.y + (double)x.y * v.x;
      }
  }
  red[t] = s;
  for (int k = 0; k < kMaxR; ++k) {
    accr[t][k] = ar[k];
    acci[t][k] = ai[k];
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      red[t] += red[t + o];
      for (int k = 0; k < r; ++k) {
        accr[t][k] += accr[t + o][k];
        acci[t][k] += acci[t + o][k];
      }
    }
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  if (t == 0) norms[m] = (float)nrm;
  if (V && t < r) dhr[(size_t)m * r + t] = cf{(float)(accr[0][t] * inv), (float)(acci[0][t] * inv)};
  for (int l = t; l < L; l += 256) dn[(size_t)m * L + l] = cf{(float)(d[l].x * inv), (float)(d[l].y * inv)};
}

// MFMA B operands: tile t (16 atoms), step q (5 K-steps of 4 for re, 5 for im), lane l:
//   q < 5 : Bre[k = 4q + l/16][atom 16t + l%16], Bre[:, m] = [Re dhr_m; Im dhr_m]
//   q >= 5: Bim[k][atom],                        Bim[:, m] = [-Im dhr_m; Re dhr_m]
// with k indexing [0, r) for the first half and [r, 2r) for the second (zero-padded to 20).
__global__ void k_dict_pack(const cf* __restrict__ dhr, int M, int r, int ntile, float* __restrict__ bpk) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)ntile * 640) return;
  const int t = (int)(idx / 640), q = (int)(idx % 640) / 64, l = (int)(idx % 64);
  const int m = 16 * t + l % 16;
  const int k = 4 * (q % 5) + l / 16;
  float v = 0.f;
  if (m < M && k < 2 * r) {
    const cf d = dhr[(size_t)m * r + (k < r ? k : k - r)];
    if (q < 5) v = k < r ? d.x : d.y;
    else v = k < r ? -d.y : d.x;
  }
  bpk[idx] = v;
}

// ---------------------------------------------------------------- frame reductions
// part[c][k][v] = sum_{l in chunk c} (X[l][v] - mu * G[l][v]) V[l][k]   (G optional)
__global__ __launch_bounds__(256) void k_reduce(const cf* __restrict__ X, const cf* __restrict__ Gd,
                                                const double* __restrict__ mu_ptr, float mu_const,
                                                const cf* __restrict__ V, int L, int Nv, int r, int fch,
                                                cf* __restrict__ part) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  const int l0 = c * fch, l1 = min(L, l0 + fch);
  const float mu = mu_ptr ? (float)mu_ptr[0] : mu_const;
  cf acc[kMaxR];
#pragma unroll
  for (int k = 0; k < kMaxR; ++k) acc[k] = cf{0.f, 0.f};
  if (v < Nv) {
    for (int l = l0; l < l1; ++l) {
      cf u = X[(size_t)l * Nv + v];
      if (Gd) {
        const cf gv = Gd[(size_t)l * Nv + v];
        u.x -= mu * gv.x;
        u.y -= mu * gv.y;
      }
#pragma unroll
      for (int k = 0; k < kMaxR; ++k)
        if (k < r) {
          const cf w = V[(size_t)l * r + k];
          acc[k].x += u.x * w.x - u.y * w.y;
          acc[k].y += u.x * w.y + u.y * w.x;
        }
    }
#pragma unroll
    for (int k = 0; k < kMaxR; ++k)
      if (k < r) part[((size_t)c * r + k) * Nv + v] = acc[k];
  }
}

// The same partial sums without G, on MFMA: D = V_c^T X_c per chunk c, with one wave per 16
// voxels. K-step = 4 frames; lane l supplies A[k = l % 16][frame l / 16] = V[frame][k] and
// B[frame l / 16][voxel l % 16] = X[frame][v0 + l % 16] (16 consecutive voxels of a frame per
// quarter-wave), and ends with components 4 (l / 16) + e of voxel v0 + l % 16. Complex from four
// real products: Re = Vr Xr - Vi Xi, Im = Vr Xi + Vi Xr.
typedef float f32x4r __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_reduce_mfma(const cf* __restrict__ X, const cf* __restrict__ V, int L, int Nv,
                                                     int r, int fch, cf* __restrict__ part) {
  const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
  const int v0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  const int c = blockIdx.y;
  const int l0 = c * fch, l1 = min(L, l0 + fch);
  const bool vv = v0 + m < Nv, kv = m < r;
  f32x4r dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
  for (int f = l0; f < l1; f += 32) {   // 8 K-steps: all loads issued before their MFMAs
    cf x[8], vk[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int fr = f + 4 * q + kk;
      const bool fv = fr < l1;
      x[q] = fv && vv ? X[(size_t)fr * Nv + v0 + m] : cf{0.f, 0.f};
      vk[q] = fv && kv ? V[(size_t)fr * r + m] : cf{0.f, 0.f};
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      dr = __builtin_amdgcn_mfma_f32_16x16x4f32(vk[q].x, x[q].x, dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_16x16x4f32(vk[q].x, x[q].y, di, 0, 0, 0);
      dr = __builtin_amdgcn_mfma_f32_16x16x4f32(-vk[q].y, x[q].y, dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_16x16x4f32(vk[q].y, x[q].x, di, 0, 0, 0);
    }
  }
  if (vv) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * kk + e;
      if (k < r) part[((size_t)c * r + k) * Nv + v0 + m] = cf{dr[e], di[e]};
    }
  }
}

// alpha[v][k] = sum_c part[c][k][v] (fixed order). One thread per voxel: the reads of part are
// coalesced over v, and the thread writes its r contiguous values.
__global__ void k_reduce_finish(const cf* __restrict__ part, int nch, int Nv, int r, cf* __restrict__ alpha) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= Nv) return;
  for (int k = 0; k < r; ++k) {
    cf s = {0.f, 0.f};
    for (int c = 0; c < nch; ++c) s = cadd(s, part[((size_t)c * r + k) * Nv + v]);
    alpha[(size_t)v * r + k] = s;
  }
}

// Z[l][v] = sum_k beta[v][k] conj(V[l][k])
__global__ __launch_bounds__(256) void k_expand(const cf* __restrict__ beta, const cf* __restrict__ V, int L, int Nv,
                                                int r, int fch, cf* __restrict__ Z) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= Nv) return;
  cf b[kMaxR];
#pragma unroll
  for (int k = 0; k < kMaxR; ++k) b[k] = k < r ? beta[(size_t)v * r + k] : cf{0.f, 0.f};
  const int l0 = blockIdx.y * fch, l1 = min(L, l0 + fch);
  for (int l = l0; l < l1; ++l) {
    cf z = {0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kMaxR; ++k)
      if (k < r) {
        const cf w = V[(size_t)l * r + k];
        z.x += b[k].x * w.x + b[k].y * w.y;
        z.y += b[k].y * w.x - b[k].x * w.y;
      }
    Z[(size_t)l * Nv + v] = z;
  }
}

// The same expansion on MFMA (r <= 16): per wave 16 voxels and a range of frames, each 16-frame
// tile D[frame][voxel] = conj(V) beta^T with K = r in steps of 4. Lane l supplies
// A[frame l % 16][k = 4 s + l / 16] = conj(V[frame][k]) and B[k][voxel l % 16] = beta[v0 + l % 16][k]
// (held in registers for all frames), and ends with frames 4 (l / 16) + e of voxel v0 + l % 16: each
// store instruction writes 16 consecutive voxels of 4 frames.
// Re = Vr br + Vi bi, Im = Vr bi - Vi br.
__global__ __launch_bounds__(256) void k_expand_mfma(const cf* __restrict__ beta, const cf* __restrict__ V, int L,
                                                     int Nv, int r, int fch, cf* __restrict__ Z) {
  const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
  const int v0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  const bool vv = v0 + m < Nv;
  float br[4], bi[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 4 * st + kk;
    const cf b = vv && k < r ? beta[(size_t)(v0 + m) * r + k] : cf{0.f, 0.f};
    br[st] = b.x;
    bi[st] = b.y;
  }
  const int nst = (r + 3) / 4;
  const int l0 = blockIdx.y * fch, l1 = min(L, l0 + fch);
  for (int f0 = l0; f0 < l1; f0 += 16) {
    const int fa = f0 + m;   // A row (frame) of this lane
    f32x4r dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      if (st < nst) {   // uniform
        const int k = 4 * st + kk;
        const cf w = fa < l1 && k < r ? V[(size_t)fa * r + k] : cf{0.f, 0.f};
        dr = __builtin_amdgcn_mfma_f32_16x16x4f32(w.x, br[st], dr, 0, 0, 0);
        di = __builtin_amdgcn_mfma_f32_16x16x4f32(w.x, bi[st], di, 0, 0, 0);
        dr = __builtin_amdgcn_mfma_f32_16x16x4f32(w.y, bi[st], dr, 0, 0, 0);
        di = __builtin_amdgcn_mfma_f32_16x16x4f32(-w.y, br[st], di, 0, 0, 0);
      }
    }
    if (vv) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int f = f0 + 4 * kk + e;
        if (f < l1) Z[(size_t)f * Nv + v0 + m] = cf{dr[e], di[e]};
      }
    }
  }
}

// beta = aU - c * Y  (c = mu * lam1 from device scalars: c = s[0] * s[1] * scale)
__global__ void k_axpy_scal(const cf* __restrict__ aU, const cf* __restrict__ Y, const double* __restrict__ s0,
                            const double* __restrict__ s1, double scale, long n, cf* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float c = (float)(s0[0] * s1[0] * scale);
  out[i] = cf{aU[i].x - c * Y[i].x, aU[i].y - c * Y[i].y};
}

// beta = aX - mu (aG + lam1 Y): the projected gradient step in the coefficient space, with
// aX = X V, aG = (A^H r) V, Y = S_L(X V) and mu, lam1 from device scalars
__global__ void k_grad_coef(const cf* __restrict__ aX, const cf* __restrict__ aG, const cf* __restrict__ Y,
                            const double* __restrict__ mu, const double* __restrict__ lam1, long n,
                            cf* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float m = (float)mu[0], c = (float)(mu[0] * lam1[0]);
  out[i] = cf{aX[i].x - m * aG[i].x - c * Y[i].x, aX[i].y - m * aG[i].y - c * Y[i].y};
}

// ---------------------------------------------------------------- subspace match (MFMA)
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct Best {
  float s;   // |<dhr_m, alpha>|^2
  int m;
};

__device__ inline bool better(float s, int m, float bs, int bm) { return s > bs || (s == bs && m < bm); }

// Block: 64 voxels, 4 waves. Each wave keeps the 4 row tiles of 16 voxels and takes the atom
// tiles t = w (mod 4); per atom tile of 16 it issues 4 x (5 + 5) MFMAs (real and imaginary parts
// of the complex products) and folds the squared magnitudes into per-lane running maxima. A
// butterfly over the 16 lanes that share a row gives each wave's arg-max, and the four waves'
// results meet in LDS (ties to the lowest atom throughout). Four waves per SIMD let one wave's
// score updates run under another's MFMAs. Atoms past M in the last tile are zero in the packed
// operands: they score 0 and lose every tie to a real atom of lower index, so they need no mask.
// Re<dhr_m, alpha> of the winner alone is formed at the end from alpha and dhr_m. A voxel whose
// alpha holds a NaN scores NaN everywhere and gets atom 0 (rho 0, score 0), never an index
// outside the dictionary.
__global__ __launch_bounds__(256, 4) void k_match_sub(const cf* __restrict__ alpha, int Nv, int r,
                                                   const float* __restrict__ bpk, const cf* __restrict__ dhr,
                                                   int ntile, int M,
                                                   const float* __restrict__ norms, const float* __restrict__ lut,
                                                   int nparam, int* __restrict__ idx_out, float* __restrict__ rho_out,
                                                   float* __restrict__ score_out, float* __restrict__ params_out) {
  __shared__ float ws_s[4][64];
  __shared__ int ws_m[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int vbase = blockIdx.x * 64;
  const int row = lane % 16, kq = lane / 16;
  // A operands: a[rt][q] = A[v = vbase + 16 rt + row][k = 4q + kq], A row = [Re alpha, Im alpha]
  float a[4][5];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    const int v = vbase + 16 * rt + row;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const int k = 4 * q + kq;
      float x = 0.f;
      if (v < Nv && k < 2 * r) {
        const cf c = alpha[(size_t)v * r + (k < r ? k : k - r)];
        x = k < r ? c.x : c.y;
      }
      a[rt][q] = x;
    }
  }
  Best best[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) best[rt][i] = Best{-1.f, 0x7fffffff};
  float b[10], bn[10];
  if (w < ntile) {
#pragma unroll
    for (int q = 0; q < 10; ++q) b[q] = bpk[((size_t)w * 10 + q) * 64 + lane];
  }
  for (int t = w; t < ntile; t += 4) {
    if (t + 4 < ntile) {
#pragma unroll
      for (int q = 0; q < 10; ++q) bn[q] = bpk[((size_t)(t + 4) * 10 + q) * 64 + lane];
    }
    const int m = 16 * t + row;   // the atom (column) this lane's outputs belong to
    // K-steps outer, row tiles inner: eight independent accumulation chains in flight
    f32x4 cre[4], cim[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      cre[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
      cim[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        cre[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][q], b[q], cre[rt], 0, 0, 0);
        cim[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][q], b[5 + q], cim[rt], 0, 0, 0);
      }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float s = cre[rt][i] * cre[rt][i] + cim[rt][i] * cim[rt][i];
        if (s > best[rt][i].s) best[rt][i] = Best{s, m};
      }
#pragma unroll
    for (int q = 0; q < 10; ++q) b[q] = bn[q];
  }
  // reduce over the 16 lanes that hold the same output rows (lane % 16 = atom column)
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Best bb = best[rt][i];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const float os = __shfl_xor(bb.s, off);
        const int om = __shfl_xor(bb.m, off);
        if (better(os, om, bb.s, bb.m)) bb = Best{os, om};
      }
      if (row == 0) {
        const int vl = 16 * rt + 4 * kq + i;   // output row of value i
        ws_s[w][vl] = bb.s;
        ws_m[w][vl] = bb.m;
      }
    }
  __syncthreads();
  if (w == 0) {
    Best bb{ws_s[0][lane], ws_m[0][lane]};
#pragma unroll
    for (int q = 1; q < 4; ++q)
      if (better(ws_s[q][lane], ws_m[q][lane], bb.s, bb.m)) bb = Best{ws_s[q][lane], ws_m[q][lane]};
    const int v = vbase + lane;
    if (v < Nv) {
      // every score of a voxel is NaN only when its alpha holds a NaN: then no comparison
      // succeeded and the sentinel stands; such a voxel is given atom 0
      const int m = bb.m < M ? bb.m : 0;
      idx_out[v] = m;
      const float nrm = norms[m];
      if (rho_out) {
        float re = 0.f;   // Re<dhr_m, alpha_v>
        for (int k = 0; k < r; ++k) {
          const cf d = dhr[(size_t)m * r + k], x = alpha[(size_t)v * r + k];
          re = fmaf(d.x, x.x, re);
          re = fmaf(d.y, x.y, re);
        }
        rho_out[v] = nrm > 0.f ? fmaxf(re / nrm, 0.f) : 0.f;
      }
      if (score_out) score_out[v] = sqrtf(fmaxf(bb.s, 0.f));
      if (params_out)
        for (int p = 0; p < nparam; ++p) params_out[(size_t)v * nparam + p] = lut[(size_t)m * nparam + p];
    }
  }
}

// maps[3][N][N] = (T1, T2, PD) from a match result
__global__ void k_maps(const int* __restrict__ idx, const float* __restrict__ rho, const float* __restrict__ lut,
                       int nparam, int Nv, float* __restrict__ maps) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= Nv) return;
  const int m = idx[v];
  maps[v] = lut[(size_t)m * nparam + 0];
  maps[Nv + v] = lut[(size_t)m * nparam + 1];
  maps[2 * Nv + v] = rho[v];
}

// ---------------------------------------------------------------- internal API
// frame chunks of the reduction: enough blocks to fill the chip (about 2048 of 256 voxels), each
// chunk at least 16 frames; fewer chunks keep the partial sums (chunks x r x Nv) small
int reduce_chunks(int L, int Nv) {
  const int vblk = (Nv + 255) / 256;
  const int want = (2048 + vblk - 1) / vblk;
  return std::max(1, std::min(std::min(64, (L + 15) / 16), want));
}

size_t reduce_ws_bytes(int L, int Nv, int r) { return (size_t)reduce_chunks(L, Nv) * r * Nv * sizeof(cf); }

// frame chunks of a reduction: MFMA blocks take 64 voxels, so fewer chunks fill the chip (never
// more than reduce_chunks, which sizes the workspace)
int reduce_nch(int L, int Nv, bool mfma) {
  return mfma ? std::max(1, std::min(reduce_chunks(L, Nv), (int)ceil_div(2048, ceil_div(Nv, 64))))
              : reduce_chunks(L, Nv);
}

// alpha [Nv][r] = (X - mu G) V, with mu from a device scalar (G may be null)
mrf_status subspace_reduce(const cf* X, const cf* Gd, const double* mu_dev, const cf* V, int L, int Nv, int r,
                           cf* alpha, cf* part, hipStream_t s) {
  const bool mf = !Gd && r <= 16;
  const int nch = reduce_nch(L, Nv, mf);
  const int fch = (L + nch - 1) / nch;
  if (mf)
    MRF_LAUNCH("subspace_reduce", s,
               k_reduce_mfma<<<dim3(ceil_div(Nv, 64), nch), 256, 0, s>>>(X, V, L, Nv, r, fch, part));
  else
    MRF_LAUNCH("subspace_reduce", s,
               k_reduce<<<dim3(ceil_div(Nv, 256), nch), 256, 0, s>>>(X, Gd, mu_dev, 1.0f, V, L, Nv, r, fch, part));
  MRF_LAUNCH("subspace_reduce_finish", s, k_reduce_finish<<<ceil_div(Nv, 256), 256, 0, s>>>(part, nch, Nv, r, alpha));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status subspace_expand(const cf* beta, const cf* V, int L, int Nv, int r, cf* Z, hipStream_t s) {
  const int nch = std::max(1, std::min(16, L / 32));
  const int fch = (L + nch - 1) / nch;
  if (r <= 16)
    MRF_LAUNCH("subspace_expand", s,
               k_expand_mfma<<<dim3(ceil_div(Nv, 64), nch), 256, 0, s>>>(beta, V, L, Nv, r, fch, Z));
  else
    MRF_LAUNCH("subspace_expand", s, k_expand<<<dim3(ceil_div(Nv, 256), nch), 256, 0, s>>>(beta, V, L, Nv, r, fch, Z));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status axpy_scal(const cf* aU, const cf* Y, const double* s0, const double* s1, double scale, long n, cf* out,
                     hipStream_t s) {
  MRF_LAUNCH("subspace_axpy", s, k_axpy_scal<<<ceil_div(n, 256), 256, 0, s>>>(aU, Y, s0, s1, scale, n, out));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status grad_coef(const cf* aX, const cf* aG, const cf* Y, const double* mu, const double* lam1, long n, cf* out,
                     hipStream_t s) {
  MRF_LAUNCH("subspace_axpy", s, k_grad_coef<<<ceil_div(n, 256), 256, 0, s>>>(aX, aG, Y, mu, lam1, n, out));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status match_subspace(const mrf_dict_s* D, const cf* alpha, int Nv, int* idx, float* rho, float* score,
                          float* params, hipStream_t s) {
  MRF_LAUNCH("match_subspace", s,
             k_match_sub<<<ceil_div(Nv, 64), 256, 0, s>>>(alpha, Nv, D->r, D->bpk, D->dhr, D->ntile, D->M, D->norms, D->lut,
                                                          D->nparam, idx, rho, score, params));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status maps_from_match(const mrf_dict_s* D, const int* idx, const float* rho, int Nv, float* maps, hipStream_t s) {
  MRF_LAUNCH("match_maps", s, k_maps<<<ceil_div(Nv, 256), 256, 0, s>>>(idx, rho, D->lut, D->nparam, Nv, maps));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

const cf* dict_basis(const mrf_dict_s* D) { return D->V; }
int dict_rank(const mrf_dict_s* D) { return D->r; }
int dict_frames(const mrf_dict_s* D) { return D->L; }

}  // namespace mrf

using namespace mrf;

extern "C" mrf_status mrf_dict_create(const mrf_c64* atoms, const float* lut, int M, int L, int nparam,
                                      const mrf_c64* V, int r, hipStream_t s, mrf_dict_t* out) {
  clear_error();
  MRF_REQUIRE(atoms && lut && out, MRF_INVALID_ARG, "dict_create: null argument");
  *out = nullptr;
  MRF_REQUIRE(M >= 1 && L >= 1 && nparam >= 2 && nparam <= 8, MRF_INVALID_ARG, "dict_create: need M, L >= 1 and 2 <= nparam <= 8");
  MRF_REQUIRE(!V || (r >= 1 && r <= 10), MRF_SHAPE, "dict_create: subspace rank r must be in [1, 10]");
  auto* D = new mrf_dict_s{};
  D->M = M; D->L = L; D->r = V ? r : 0; D->nparam = nparam;
  D->ntile = (M + 15) / 16;
  D->Lp = (L + 127) / 128 * 128;   // a whole number of every match form's frame chunks
  bool ok = hipMalloc(&D->lut, (size_t)M * nparam * 4) == hipSuccess && hipMalloc(&D->norms, (size_t)M * 4) == hipSuccess &&
            hipMalloc(&D->dn, (size_t)M * L * sizeof(cf)) == hipSuccess &&
            hipMalloc(&D->d16, (size_t)M * 2 * D->Lp * 2) == hipSuccess &&
            hipMalloc(&D->d16lo, (size_t)M * 2 * D->Lp * 2) == hipSuccess &&
            hipMalloc(&D->d8, (size_t)M * 2 * D->Lp) == hipSuccess && hipMalloc(&D->s8, (size_t)M * 4) == hipSuccess;
  if (ok && V)
    ok = hipMalloc(&D->dhr, (size_t)M * r * sizeof(cf)) == hipSuccess &&
         hipMalloc(&D->bpk, (size_t)D->ntile * 640 * 4) == hipSuccess &&
         hipMalloc(&D->V, (size_t)L * r * sizeof(cf)) == hipSuccess;
  if (!ok) {
    mrf_dict_destroy(D);
    return fail(MRF_OOM, "dict_create: device allocation failed");
  }
  hipError_t e = hipMemcpyAsync(D->lut, lut, (size_t)M * nparam * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && V) e = hipMemcpyAsync(D->V, V, (size_t)L * r * sizeof(cf), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    mrf_dict_destroy(D);
    return fail(MRF_DEVICE, "dict_create: copy failed");
  }
  k_dict_prep<<<M, 256, 0, s>>>((const cf*)atoms, (const cf*)V, M, L, V ? r : 0, D->norms, D->dhr, D->dn);
  if (V) k_dict_pack<<<ceil_div((long)D->ntile * 640, 256), 256, 0, s>>>(D->dhr, M, r, D->ntile, D->bpk);
  e = hipGetLastError();
  if (e == hipSuccess && quantise_rows(D->dn, M, L, D->Lp, D->d16, D->d16lo, D->d8, D->s8, s) != MRF_OK) e = hipErrorLaunchFailure;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    mrf_dict_destroy(D);
    return fail(MRF_DEVICE, std::string("dict_create: ") + hipGetErrorString(e));
  }
  *out = D;
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_destroy(mrf_dict_t D) {
  clear_error();
  if (!D) return MRF_OK;
  hipFree(D->lut); hipFree(D->norms); hipFree(D->dhr); hipFree(D->bpk); hipFree(D->V); hipFree(D->dn);
  hipFree(D->d16); hipFree(D->d16lo); hipFree(D->d8); hipFree(D->s8);
  delete D;
  return MRF_OK;
}

extern "C" mrf_status mrf_subspace_coeffs_workspace_size(int L, int Nv, int r, size_t* bytes) {
  clear_error();
  MRF_REQUIRE(bytes && L >= 1 && Nv >= 1 && r >= 1 && r <= kMaxR, MRF_INVALID_ARG, "subspace_coeffs_workspace_size: bad argument");
  *bytes = reduce_ws_bytes(L, Nv, r);
  return MRF_OK;
}

extern "C" mrf_status mrf_subspace_coeffs(const mrf_c64* X, const mrf_c64* V, int L, int Nv, int r, mrf_c64* alpha,
                                          void* ws, size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(X && V && alpha, MRF_INVALID_ARG, "subspace_coeffs: null argument");
  MRF_REQUIRE(L >= 1 && Nv >= 1 && r >= 1 && r <= kMaxR, MRF_INVALID_ARG, "subspace_coeffs: bad sizes");
  MRF_REQUIRE(ws && ws_bytes >= reduce_ws_bytes(L, Nv, r), MRF_WORKSPACE, "subspace_coeffs: workspace too small");
  return subspace_reduce((const cf*)X, nullptr, nullptr, (const cf*)V, L, Nv, r, (cf*)alpha, (cf*)ws, s);
}

// ---------------------------------------------------------------- no-allocation variant
// The partial sums of mrf_subspace_coeffs_noalloc live in this file-scope device array (one copy
// per GPU, held until the process ends). Host code never passes the array's name to a kernel or a
// copy: on the host that name is only a stand-in, so its device address is looked up once per
// device (hipGetSymbolAddress with the device current) and kept in g_scratch_dev.
constexpr size_t kCoeffScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) char scratch[kCoeffScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;   // by device ordinal; null until looked up

mrf_status scratch_address(void** out) {
  int dev = -1;
  MRF_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    MRF_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MRF_REQUIRE(p, MRF_DEVICE, "subspace_coeffs_noalloc: no device address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return MRF_OK;
}
}  // namespace

extern "C" mrf_status mrf_subspace_coeffs_noalloc(const mrf_c64* X, const mrf_c64* V, int L, int Nv, int r,
                                                  mrf_c64* alpha, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(X && V && alpha, MRF_INVALID_ARG, "subspace_coeffs_noalloc: null argument");
  MRF_REQUIRE(L >= 1 && Nv >= 1 && r >= 1 && r <= kMaxR, MRF_INVALID_ARG, "subspace_coeffs_noalloc: bad sizes");
  // the partial sums the reduction writes: chunks x r x Nv (what mrf_subspace_coeffs uses of its workspace)
  const size_t need = (size_t)reduce_nch(L, Nv, true) * r * Nv * sizeof(cf);
  MRF_REQUIRE(need <= kCoeffScratchBytes, MRF_WORKSPACE,
              "subspace_coeffs_noalloc: the partial sums exceed the 16 MiB scratch array (chunks x r x Nv x 8 bytes)");
  void* part = nullptr;
  mrf_status e = scratch_address(&part);
  if (e) return e;
  return subspace_reduce((const cf*)X, nullptr, nullptr, (const cf*)V, L, Nv, r, (cf*)alpha, (cf*)part, s);
}

extern "C" mrf_status mrf_subspace_project(const mrf_c64* U, const mrf_c64* V, int L, int Nv, int r, mrf_c64* Z,
                                           void* ws, size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(U && V && Z, MRF_INVALID_ARG, "subspace_project: null argument");
  MRF_REQUIRE(L >= 1 && Nv >= 1 && r >= 1 && r <= kMaxR, MRF_INVALID_ARG, "subspace_project: bad sizes");
  const size_t need = reduce_ws_bytes(L, Nv, r) + (size_t)Nv * r * sizeof(cf);
  MRF_REQUIRE(ws && ws_bytes >= need, MRF_WORKSPACE, "subspace_project: workspace too small");
  cf* alpha = (cf*)((char*)ws + reduce_ws_bytes(L, Nv, r));
  mrf_status st = subspace_reduce((const cf*)U, nullptr, nullptr, (const cf*)V, L, Nv, r, alpha, (cf*)ws, s);
  if (st != MRF_OK) return st;
  return subspace_expand(alpha, (const cf*)V, L, Nv, r, (cf*)Z, s);
}

extern "C" mrf_status mrf_dict_match_subspace(mrf_dict_t D, const mrf_c64* alpha, int Nv, int32_t* idx, float* rho,
                                              float* score, float* params, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(D && alpha && idx, MRF_INVALID_ARG, "dict_match_subspace: null argument");
  MRF_REQUIRE(D->r > 0, MRF_INVALID_ARG, "dict_match_subspace: dictionary was created without a basis");
  MRF_REQUIRE(Nv >= 1, MRF_INVALID_ARG, "dict_match_subspace: Nv must be >= 1");
  return match_subspace(D, (const cf*)alpha, Nv, idx, rho, score, params, s);
}
