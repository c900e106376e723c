// Learned matching: an MLP from subspace coefficients to (log T1, log T2), trained and run on the
// GPU, with a residual gate that sends poorly explained voxels to the exhaustive match.
//
// The paper's matching is the exhaustive search of eq. (5) (Sec. II-B); it cites learned
// signal-to-parameter mappings as related work. This form of it is the library's own:
//   features  alpha = x V (r complex), alpha / ||alpha||, rotated so that alpha_0 is real >= 0,
//             z = (Re alpha, Im alpha) in R^{2r}
//   network   h_l = relu(W_l h_{l-1} + b_l) (hidden layers), y = W_L h_{L-1} + b_L, y the
//             standardised (log T1, log T2): (log T - mean) / std over the dictionary atoms
//   loss      mean over batch and outputs of (y - t)^2; Adam with bias correction, cosine lr
//   batches   sample i of step s: Philox4x32-10 with key = seed and counter (i, s, c, 0) gives the
//             atom m = mulhi32(u0, M), the phase 2 pi (u1 + 1/2) 2^-32, the SNR uniform in
//             [snr_lo, snr_hi] dB from u2, and (c = 1, 2, ...) Box-Muller normals for complex noise
//             of variance 10^(-SNR/10) / L per coefficient (exact in distribution in the subspace:
//             the columns of V are orthonormal); alpha = exp(i phase) d_m V / ||d_m|| + noise
//   gate      k* = the kept grid atom nearest to the prediction in Euclidean distance on
//             (log T1, log T2), ties to the lower index; residual =
//             1 - |<d_k* V / ||d_k*||, alpha / ||alpha||>|; residual > theta -> exhaustive match.
//
// GEMMs: one MFMA kernel with 64 x 64 output tiles (4 waves of 32 x 32), K staged through LDS in
// chunks of 32 from either operand layout (K-contiguous or K-strided), in FP32
// (v_mfma_f32_16x16x4f32) or BF16 (operands rounded to nearest-even in registers,
// v_mfma_f32_16x16x32_bf16), FP32 accumulation; epilogues for bias, ReLU and the ReLU mask of the
// backward pass; split-K with a fixed-order reduction for the weight gradients (K = batch), which
// in the BF16 step one launch takes for all layers together with the Adam step.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "dict.hpp"
#include "philox.hpp"

struct mrf_mlp_s {
  int nin, hid, nhl, nout;      // input width, hidden width, hidden layers, outputs
  int nl;                       // layers = nhl + 1
  std::vector<size_t> offW, offb;
  std::vector<int> lin, lout;
  size_t np;                    // parameter count
  float *p, *g, *m, *v;         // parameters, gradients, Adam moments (flat, FP32)
  int t;                        // Adam step count
  double *stats;                // device [4]: mean(log T1), mean(log T2), std(log T1), std(log T2)
  bool have_stats;
  // log-spaced (T1, T2) grid for the gate
  int n1, n2;
  double l1_0, dl1, l2_0, dl2;
  int *gidx, *i2max;            // [n1][n2] atom index (or -1), [n1] largest kept T2 index
  int gmax;                     // largest atom index in the grid
};

namespace mrf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxR = 16;

// z [B][2r] features and t [B][2] standardised targets of a synthetic training batch; m [B].
// The rank R is a template parameter so that the noise and coefficient arrays stay in registers.
struct SynthArgs {
  const cf* dhr;
  int M;
  const float* lut;
  int nparam;
  const double* stats;
  unsigned k0, k1, step;
  int B;
  float snr_lo, snr_hi, L;
  float* z;
  float* t;
  int* mo;
};
template <int R>
__device__ inline void synth_one(const SynthArgs& a, int i) {
  if (i >= a.B) return;
  const unsigned k0 = a.k0, k1 = a.k1, step = a.step;
  const u4 u = philox(u4{(unsigned)i, step, 0u, 0u}, k0, k1);
  const int m = (int)(((unsigned long long)u.x * (unsigned)a.M) >> 32);
  const float phi = 6.283185307179586f * u01(u.y);
  const float snr = a.snr_lo + (a.snr_hi - a.snr_lo) * u01(u.z);
  const float sig = sqrtf(powf(10.f, -snr / 10.f) / a.L) * 0.70710678118654752f;
  constexpr int NC = (2 * R + 3) / 4;
  float gs[4 * NC];
#pragma unroll
  for (int c = 1; c <= NC; ++c) {
    const u4 v = philox(u4{(unsigned)i, step, (unsigned)c, 0u}, k0, k1);
    const float r0 = sqrtf(-2.f * logf(u01(v.x))), a0 = 6.283185307179586f * u01(v.y);
    const float r1 = sqrtf(-2.f * logf(u01(v.z))), a1 = 6.283185307179586f * u01(v.w);
    gs[4 * (c - 1) + 0] = r0 * cosf(a0);
    gs[4 * (c - 1) + 1] = r0 * sinf(a0);
    gs[4 * (c - 1) + 2] = r1 * cosf(a1);
    gs[4 * (c - 1) + 3] = r1 * sinf(a1);
  }
  const float cp = cosf(phi), sp = sinf(phi);
  float ar[R], ai[R], nrm = 0.f;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const cf d = a.dhr[(size_t)m * R + k];
    ar[k] = cp * d.x - sp * d.y + gs[k] * sig;
    ai[k] = sp * d.x + cp * d.y + gs[R + k] * sig;
    nrm += ar[k] * ar[k] + ai[k] * ai[k];
  }
  nrm = sqrtf(nrm);
  const float a0m = sqrtf(ar[0] * ar[0] + ai[0] * ai[0]);
  const float c0 = a0m > 0.f ? ar[0] / a0m : 1.f, s0 = a0m > 0.f ? -ai[0] / a0m : 0.f;   // exp(-i angle)
  const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    a.z[(size_t)i * 2 * R + k] = (ar[k] * c0 - ai[k] * s0) * inv;
    a.z[(size_t)i * 2 * R + R + k] = (ar[k] * s0 + ai[k] * c0) * inv;
  }
  const float* lu = a.lut + (size_t)m * a.nparam;
  a.t[(size_t)i * 2 + 0] = (float)((log((double)lu[0]) - a.stats[0]) / a.stats[2]);
  a.t[(size_t)i * 2 + 1] = (float)((log((double)lu[1]) - a.stats[1]) / a.stats[3]);
  if (a.mo) a.mo[i] = m;
}
template <int R>
__global__ __launch_bounds__(256) void k_synth(SynthArgs a) {
  synth_one<R>(a, blockIdx.x * 256 + threadIdx.x);
}

// launches k_synth<r> for the dictionary's rank (1 .. kMaxR)
template <int R = 1>
static void launch_synth(int r, dim3 grid, hipStream_t s, const SynthArgs& a) {
  if constexpr (R <= kMaxR) {
    if (r == R) k_synth<R><<<grid, 256, 0, s>>>(a);
    else launch_synth<R + 1>(r, grid, s, a);
  }
}

// features of measured coefficients alpha [Nv][r]
__global__ __launch_bounds__(256) void k_features(const cf* __restrict__ alpha, int Nv, int r, float* __restrict__ z) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= Nv) return;
  const cf* a = alpha + (size_t)i * r;
  float nrm = 0.f;
  for (int k = 0; k < r; ++k) nrm += a[k].x * a[k].x + a[k].y * a[k].y;
  nrm = sqrtf(nrm);
  const float a0m = sqrtf(a[0].x * a[0].x + a[0].y * a[0].y);
  const float c0 = a0m > 0.f ? a[0].x / a0m : 1.f, s0 = a0m > 0.f ? -a[0].y / a0m : 0.f;
  const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
  for (int k = 0; k < r; ++k) {
    z[(size_t)i * 2 * r + k] = (a[k].x * c0 - a[k].y * s0) * inv;
    z[(size_t)i * 2 * r + r + k] = (a[k].x * s0 + a[k].y * c0) * inv;
  }
}

// mean and standard deviation of log T1, log T2 over the atoms (one block, fixed order)
__global__ __launch_bounds__(256) void k_target_stats(const float* __restrict__ lut, int M, int nparam,
                                                      double* __restrict__ stats) {
  __shared__ double red[4][256];
  const int t = threadIdx.x;
  double s1 = 0, s2 = 0, q1 = 0, q2 = 0;
  for (int m = t; m < M; m += 256) {
    const double a = log((double)lut[(size_t)m * nparam]), b = log((double)lut[(size_t)m * nparam + 1]);
    s1 += a; s2 += b; q1 += a * a; q2 += b * b;
  }
  red[0][t] = s1; red[1][t] = s2; red[2][t] = q1; red[3][t] = q2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o)
      for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + o];
    __syncthreads();
  }
  if (t == 0) {
    const double m1 = red[0][0] / M, m2 = red[1][0] / M;
    stats[0] = m1;
    stats[1] = m2;
    stats[2] = sqrt(fmax(red[2][0] / M - m1 * m1, 1e-300));
    stats[3] = sqrt(fmax(red[3][0] / M - m2 * m2, 1e-300));
  }
}

// ------------------------------------------------------------------ GEMM
// C[m][n] (+)= sum_k A(m, k) B(k, n);  A(m, k) = A[m lda + k] (AK) or A[k lda + m] (AM);
// B(k, n) = B[n ldb + k] (BK) or B[k ldb + n] (BN). Split-K slice z covers k in
// [z ks, (z + 1) ks) and writes C + z M ldc.
enum { LAY_K = 0, LAY_MN = 1 };
enum { EPI_STORE = 0, EPI_BIAS_RELU = 1, EPI_BIAS = 2, EPI_MASK = 3 };
constexpr int kG = 64, kGK = 32;

__device__ inline unsigned bf16pair(float a, float b) {
  const unsigned ua = __float_as_uint(a), ub = __float_as_uint(b);
  const unsigned ra = (ua + 0x7fffu + ((ua >> 16) & 1u)) >> 16, rb = (ub + 0x7fffu + ((ub >> 16) & 1u)) >> 16;
  return ra | (rb << 16);
}

template <bool BF16, int ALAY, int BLAY, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, const float* __restrict__ mask, int mld,
                                              int ks) {
  __shared__ float As[kG][kGK + 1], Bs[kG][kGK + 1];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wm = w >> 1, wn = w & 1, q = lane >> 4, n16 = lane & 15;
  const int n0 = blockIdx.x * kG, m0 = blockIdx.y * kG;
  const int kb = blockIdx.z * ks, ke = min(K, kb + ks);
  C += (size_t)blockIdx.z * M * ldc;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kG * kGK / 256; ++j) {
      const int idx = tid + 256 * j;
      int r, c;
      if (ALAY == LAY_K) { r = idx / kGK; c = idx % kGK; }
      else { c = idx / kG; r = idx % kG; }
      const int m = m0 + r, k = k0 + c;
      As[r][c] = (m < M && k < ke) ? (ALAY == LAY_K ? A[(size_t)m * lda + k] : A[(size_t)k * lda + m]) : 0.f;
      if (BLAY == LAY_K) { r = idx / kGK; c = idx % kGK; }
      else { c = idx / kG; r = idx % kG; }
      const int n = n0 + r, k2 = k0 + c;
      Bs[r][c] = (n < N && k2 < ke) ? (BLAY == LAY_K ? B[(size_t)n * ldb + k2] : B[(size_t)k2 * ldb + n]) : 0.f;
    }
    __syncthreads();
    if constexpr (BF16) {
      bf16x8 av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float* s = &As[wm * 32 + a * 16 + n16][8 * q];
        const unsigned u[4] = {bf16pair(s[0], s[1]), bf16pair(s[2], s[3]), bf16pair(s[4], s[5]), bf16pair(s[6], s[7])};
        av[a] = __builtin_bit_cast(bf16x8, make_uint4(u[0], u[1], u[2], u[3]));
        const float* t = &Bs[wn * 32 + a * 16 + n16][8 * q];
        const unsigned v[4] = {bf16pair(t[0], t[1]), bf16pair(t[2], t[3]), bf16pair(t[4], t[5]), bf16pair(t[6], t[7])};
        bv[a] = __builtin_bit_cast(bf16x8, make_uint4(v[0], v[1], v[2], v[3]));
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    } else {
#pragma unroll
      for (int s = 0; s < kGK / 4; ++s) {
        float av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          av[a] = As[wm * 32 + a * 16 + n16][4 * s + q];
          bv[a] = Bs[wn * 32 + a * 16 + n16][4 * s + q];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + wm * 32 + a * 16 + 4 * q + i, n = n0 + wn * 32 + b * 16 + n16;
        if (m < M && n < N) {
          float v = acc[a][b][i];
          if (EPI == EPI_BIAS_RELU) v = fmaxf(v + bias[n], 0.f);
          else if (EPI == EPI_BIAS) v += bias[n];
          else if (EPI == EPI_MASK) v = mask[(size_t)m * mld + n] > 0.f ? v : 0.f;
          C[(size_t)m * ldc + n] = v;
        }
      }
}

// BF16 GEMM with the same contract as k_gemm<true, ...>, software-pipelined: 64 x 64 tiles with
// K steps of 64; the next step's operands are loaded into registers while the MFMAs of this one
// run, then converted to BF16 once and stored to the other half of a double-buffered LDS tile (one
// barrier per step). A lane's 8 consecutive k values of a row are one 16-byte LDS read.
constexpr int kGB = 64, kGBK = 64, kGBP = kGBK + 8;   // tile, K step, LDS row pitch (bf16)
__device__ inline unsigned short bf16_rne(float a) {
  const unsigned u = __float_as_uint(a);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// With asum (A laid out [k][m] only), the blocks of the first column tile also write the FP32
// sums over their k slice of A's rows, asum[z M + m] = sum_k A(m, k): the bias gradient of the
// weight-gradient product, in a fixed order (per thread in k order, then the four waves in order).
// One operand tile (64 rows x 64 k) of a step: loads into registers (float4 where the layout,
// the leading dimension and the extents allow: V4), then BF16 into LDS.
template <int LAY, bool V4>
struct TileOp {
  static constexpr int NL = V4 ? kGB * kGBK / 1024 : kGB * kGBK / 256;
  float v[V4 ? 4 * NL : NL];
  __device__ inline void load(const float* __restrict__ X, int ld, int row0, int rows, int k0, int ke, int tid) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      if (V4) {
        const int idx = tid + 256 * j;
        int r, c;
        if (LAY == LAY_K) { r = idx >> 4; c = (idx & 15) << 2; }
        else { c = idx >> 4; r = (idx & 15) << 2; }
        const int row = row0 + r, k = k0 + c;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < rows && k < ke)
          x = *(const float4*)(LAY == LAY_K ? X + (size_t)row * ld + k : X + (size_t)k * ld + row);
        v[4 * j] = x.x; v[4 * j + 1] = x.y; v[4 * j + 2] = x.z; v[4 * j + 3] = x.w;
      } else {
        const int idx = tid + 256 * j;
        int r, c;
        if (LAY == LAY_K) { r = idx / kGBK; c = idx % kGBK; }
        else { c = idx / kGB; r = idx % kGB; }
        const int row = row0 + r, k = k0 + c;
        v[j] = (row < rows && k < ke) ? (LAY == LAY_K ? X[(size_t)row * ld + k] : X[(size_t)k * ld + row]) : 0.f;
      }
    }
  }
  __device__ inline void store(unsigned short (*Xs)[kGBP], int tid) const {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int idx = tid + 256 * j;
      if (V4) {
        if (LAY == LAY_K) {
          const int r = idx >> 4, c = (idx & 15) << 2;
          *(uint2*)&Xs[r][c] = make_uint2(bf16pair(v[4 * j], v[4 * j + 1]), bf16pair(v[4 * j + 2], v[4 * j + 3]));
        } else {
          const int c = idx >> 4, r = (idx & 15) << 2;
#pragma unroll
          for (int i = 0; i < 4; ++i) Xs[r + i][c] = bf16_rne(v[4 * j + i]);
        }
      } else {
        int r, c;
        if (LAY == LAY_K) { r = idx / kGBK; c = idx % kGBK; }
        else { c = idx / kGB; r = idx % kGB; }
        Xs[r][c] = bf16_rne(v[j]);
      }
    }
  }
};

// Adam with bias correction for one parameter: c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
struct AdamArgs {
  float lr, b1, b2, eps, c1, c2;
};
__device__ inline void adam_update(float& p, float& m, float& v, float g, const AdamArgs& a) {
  const float mi = a.b1 * m + (1.f - a.b1) * g;
  const float vi = a.b2 * v + (1.f - a.b2) * g * g;
  m = mi;
  v = vi;
  p -= a.lr * (mi * a.c1) / (sqrtf(vi * a.c2) + a.eps);
}

struct GemmLds {
  unsigned short As[2][kGB][kGBP];
  unsigned short Bs[2][kGB][kGBP];
  float sred[4][kGB];
};
// output tile (bx, by) of split-K slice bz
template <int ALAY, int BLAY, int EPI, bool AV4, bool BV4>
__device__ inline void gemm_bf16_tile(int M, int N, int K, const float* __restrict__ A, int lda,
                                      const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                      const float* __restrict__ bias, const float* __restrict__ mask, int mld, int ks,
                                      float* __restrict__ asum, int bx, int by, int bz, GemmLds& sm) {
  auto& As = sm.As;
  auto& Bs = sm.Bs;
  auto& sred = sm.sred;
  // the column sums read A's scalar tile (r = lane for every element): only without AV4
  const bool do_sum = ALAY == LAY_MN && !AV4 && asum && bx == 0;
  float rsum = 0.f;   // this thread's row (m0 + lane) of A over its k values
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wm = w >> 1, wn = w & 1, q = lane >> 4, n16 = lane & 15;
  const int n0 = bx * kGB, m0 = by * kGB;
  const int kb = bz * ks, ke = min(K, kb + ks);
  C += (size_t)bz * M * ldc;
  TileOp<ALAY, AV4> ta;
  TileOp<BLAY, BV4> tb;
  auto load = [&](int k0) {
    ta.load(A, lda, m0, M, k0, ke, tid);
    tb.load(B, ldb, n0, N, k0, ke, tid);
  };
  auto store = [&](int buf) {
    if (!AV4 && ALAY == LAY_MN && do_sum) {
#pragma unroll
      for (int j = 0; j < TileOp<ALAY, AV4>::NL; ++j) rsum += ta.v[j];   // r = lane for every j
    }
    ta.store(As[buf], tid);
    tb.store(Bs[buf], tid);
  };
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  load(kb);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += kGBK) {
    const bool more = k0 + kGBK < ke;
    if (more) load(k0 + kGBK);
#pragma unroll
    for (int kk = 0; kk < kGBK; kk += 32) {
      bf16x8 av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        av[a] = *(const bf16x8*)&As[buf][wm * 32 + a * 16 + n16][kk + 8 * q];
        bv[a] = *(const bf16x8*)&Bs[buf][wn * 32 + a * 16 + n16][kk + 8 * q];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (ALAY == LAY_MN && do_sum) {
    sred[w][lane] = rsum;
    __syncthreads();
    if (w == 0 && m0 + lane < M)
      asum[(size_t)bz * M + m0 + lane] = (sred[0][lane] + sred[1][lane]) + (sred[2][lane] + sred[3][lane]);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + wm * 32 + a * 16 + 4 * q + i, n = n0 + wn * 32 + b * 16 + n16;
        if (m < M && n < N) {
          float v = acc[a][b][i];
          if (EPI == EPI_BIAS_RELU) v = fmaxf(v + bias[n], 0.f);
          else if (EPI == EPI_BIAS) v += bias[n];
          else if (EPI == EPI_MASK) v = mask[(size_t)m * mld + n] > 0.f ? v : 0.f;
          C[(size_t)m * ldc + n] = v;
        }
      }
}

template <int ALAY, int BLAY, int EPI, bool AV4, bool BV4>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const float* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                   int ldc, const float* __restrict__ bias,
                                                   const float* __restrict__ mask, int mld, int ks,
                                                   float* __restrict__ asum) {
  __shared__ __align__(16) GemmLds sm;
  gemm_bf16_tile<ALAY, BLAY, EPI, AV4, BV4>(M, N, K, A, lda, B, ldb, C, ldc, bias, mask, mld, ks, asum, blockIdx.x,
                                            blockIdx.y, blockIdx.z, sm);
}

// Operands of one product of a grouped launch, and its tile grid gx x gy (x gz slices)
struct GemmArgs {
  int M, N, K;
  const float* A;
  int lda;
  const float* B;
  int ldb;
  float* C;
  int ldc;
  const float* mask;
  int mld, ks;
  float* asum;
  int gx, gy;
};
// A layer's two backward products in one launch: they read the same output gradient and not each
// other's results. Blocks [0, d.gx d.gy) take the backward product d (masked by the layer's ReLU),
// the rest the split-K weight-gradient product w with its bias-gradient column sums.
template <bool DA4>
__global__ __launch_bounds__(256) void k_gemm_bf16_bwd_pair(GemmArgs d, GemmArgs w) {
  __shared__ __align__(16) GemmLds sm;
  const int nd = d.gx * d.gy;
  int b = blockIdx.x;
  if (b < nd) {
    gemm_bf16_tile<LAY_K, LAY_MN, EPI_MASK, DA4, true>(d.M, d.N, d.K, d.A, d.lda, d.B, d.ldb, d.C, d.ldc, nullptr,
                                                       d.mask, d.mld, d.ks, nullptr, b % d.gx, b / d.gx, 0, sm);
  } else {
    b -= nd;
    const int nt = w.gx * w.gy, t = b % nt;
    gemm_bf16_tile<LAY_MN, LAY_MN, EPI_STORE, false, true>(w.M, w.N, w.K, w.A, w.lda, w.B, w.ldb, w.C, w.ldc, nullptr,
                                                           nullptr, 0, w.ks, w.asum, t % w.gx, t / w.gx, b / nt, sm);
  }
}

// The end of the BF16 backward pass in one launch: every weight and bias gradient is the sum of
// its split-K slices (slice order), written to g, and with adam set the Adam step follows.
// Segment k (blocks k gx .. k gx + gx - 1) holds cnt[k] parameters from offset off[k], slices
// part[k] [S][cnt[k]].
constexpr int kMaxSeg = 2 * 9;
struct GradSegs {
  int n;
  const float* part[kMaxSeg];
  long off[kMaxSeg];
  int cnt[kMaxSeg];
  int gx;                   // blocks per segment
};
__device__ inline void grad_finish_one(const GradSegs& sg, int S, float* __restrict__ g, float* __restrict__ p,
                                       float* __restrict__ m, float* __restrict__ v, const AdamArgs& ad, int adam,
                                       int k, int i) {
  if (k >= sg.n || i >= sg.cnt[k]) return;
  const float* pt = sg.part[k];
  const size_t n = (size_t)sg.cnt[k];
  float sum = 0.f;
  for (int z = 0; z < S; ++z) sum += pt[z * n + i];
  const long o = sg.off[k] + i;
  g[o] = sum;
  if (adam) {
    float pi = p[o], mi = m[o], vi = v[o];
    adam_update(pi, mi, vi, sum, ad);
    m[o] = mi;
    v[o] = vi;
    p[o] = pi;
  }
}
__global__ __launch_bounds__(256) void k_grad_finish(GradSegs sg, int S, float* __restrict__ g, float* __restrict__ p,
                                                     float* __restrict__ m, float* __restrict__ v, AdamArgs ad,
                                                     int adam) {
  grad_finish_one(sg, S, g, p, m, v, ad, adam, blockIdx.x / sg.gx, (blockIdx.x % sg.gx) * 256 + threadIdx.x);
}
// The same, and in the same launch the next training batch (blocks from sg.n sg.gx on): the batch
// buffers are free once the last weight-gradient product has read them.
template <int R>
__global__ __launch_bounds__(256) void k_grad_finish_synth(GradSegs sg, int S, float* __restrict__ g,
                                                           float* __restrict__ p, float* __restrict__ m,
                                                           float* __restrict__ v, AdamArgs ad, int adam, SynthArgs sa) {
  const int nf = sg.n * sg.gx;
  if ((int)blockIdx.x < nf)
    grad_finish_one(sg, S, g, p, m, v, ad, adam, blockIdx.x / sg.gx, (blockIdx.x % sg.gx) * 256 + threadIdx.x);
  else
    synth_one<R>(sa, (blockIdx.x - nf) * 256 + threadIdx.x);
}
template <int R = 1>
static void launch_finish_synth(int r, int grid, hipStream_t s, const GradSegs& sg, int S, float* g, float* p, float* m,
                                float* v, const AdamArgs& ad, int adam, const SynthArgs& sa) {
  if constexpr (R <= kMaxR) {
    if (r == R) k_grad_finish_synth<R><<<grid, 256, 0, s>>>(sg, S, g, p, m, v, ad, adam, sa);
    else launch_finish_synth<R + 1>(r, grid, s, sg, S, g, p, m, v, ad, adam, sa);
  }
}

// out[i] = sum_s part[s n + i] (fixed order)
__global__ __launch_bounds__(256) void k_reduce_slices(const float* __restrict__ part, int S, long n,
                                                       float* __restrict__ out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int k = 0; k < S; ++k) s += part[(size_t)k * n + i];
  out[i] = s;
}

// db[n] = sum_b G[b][n]: block per 64 columns, 4 row phases, fixed-order tree
// Column sums db[c] = sum_b G[b][c] in two fixed-order stages: block (x, y) sums rows
// y * kColRows .. of 64 columns into part[y][c] (4 row phases per column, then a fixed tree), and
// one thread per column adds the partials in order.
constexpr int kColRows = 128;
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ G, int Bn, int N, float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
  const int b0 = blockIdx.y * kColRows, b1 = min(Bn, b0 + kColRows);
  float s = 0.f;
  if (c < N)
    for (int b = b0 + ph; b < b1; b += 4) s += G[(size_t)b * N + c];
  red[ph][threadIdx.x & 63] = s;
  __syncthreads();
  if (ph == 0 && c < N)
    part[(size_t)blockIdx.y * N + c] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}
__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ part, int nch, int N, float* __restrict__ db) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  float s = 0.f;
  for (int k = 0; k < nch; ++k) s += part[(size_t)k * N + c];
  db[c] = s;
}

// g = 2 (y - t) / (B nout); per-block partial sums of (y - t)^2 into lpart; the last block to
// finish (counter *cnt, zero before the launch and reset by that block) sums the partials in block
// order into loss (and loss2 when set): the mean over batch and outputs.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t, int n, float scale,
                                              float* __restrict__ g, float* __restrict__ lpart, unsigned* __restrict__ cnt,
                                              float* __restrict__ loss, float* __restrict__ loss2) {
  __shared__ float red[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  float d = 0.f;
  if (i < n) {
    d = y[i] - t[i];
    g[i] = 2.f * d * scale;
  }
  red[threadIdx.x] = d * d;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(cnt, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  float s = 0.f;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += 256) s += lpart[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    loss[0] = red[0] * scale;
    if (loss2) loss2[0] = red[0] * scale;
    cnt[0] = 0u;
  }
}

__global__ void k_zero_u32(unsigned* __restrict__ p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, long n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float pi = p[i], mi = m[i], vi = v[i];
  adam_update(pi, mi, vi, g[i], AdamArgs{lr, b1, b2, eps, c1, c2});
  m[i] = mi;
  v[i] = vi;
  p[i] = pi;
}

// He-normal initialisation from Philox (counter (index, layer, 0x48e, 0)), zero biases
__global__ __launch_bounds__(256) void k_init(float* __restrict__ W, long n, float sd, unsigned layer, unsigned k0,
                                              unsigned k1) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const u4 u = philox(u4{(unsigned)i, layer, 0x48eu, 0u}, k0, k1);
  W[i] = sd * sqrtf(-2.f * logf(u01(u.x))) * cosf(6.283185307179586f * u01(u.y));
}

// Gate: k* = the kept grid atom nearest to the prediction exp(y * std + mean) in Euclidean distance
// on (log T1, log T2), ties to the lower atom index; then the residual and rho, and voxels above
// theta are flagged. Row a of the grid keeps T2 indices 0 .. i2max[a] (checked by set_grid), so a
// row's nearest kept point is floor(x2) or floor(x2) + 1 clamped into that range; rows are taken
// in ascending order with a strict comparison, which keeps the lower index on ties, and a row is
// skipped when its T1 distance alone reaches the best found.
__global__ __launch_bounds__(256) void k_gate(const float* __restrict__ y, const double* __restrict__ stats, int n1,
                                              int n2, double l1_0, double dl1, double l2_0, double dl2,
                                              const int* __restrict__ gidx, const int* __restrict__ i2max,
                                              const cf* __restrict__ dhr, const float* __restrict__ norms,
                                              const cf* __restrict__ alpha, int Nv, int r, float theta,
                                              int* __restrict__ idx, float* __restrict__ t12, float* __restrict__ rho,
                                              float* __restrict__ resid, int* __restrict__ fb, int* __restrict__ nfb,
                                              int* __restrict__ fblist) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= Nv) return;
  const double lt1 = (double)y[(size_t)v * 2] * stats[2] + stats[0];
  const double lt2 = (double)y[(size_t)v * 2 + 1] * stats[3] + stats[1];
  const double x2 = (lt2 - l2_0) / dl2;
  const double fl = floor(x2);
  const int blo = fl < 0.0 ? -1 : (fl >= (double)n2 ? n2 : (int)fl);
  double best = 1.0e300;
  int ba = 0, bb = 0;
  for (int a = 0; a < n1; ++a) {
    const double d1 = lt1 - (l1_0 + a * dl1);
    const double d11 = d1 * d1;
    if (d11 >= best) continue;
    const int hi = i2max[a];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int b = min(max(blo + c, 0), hi);
      const double d2 = lt2 - (l2_0 + b * dl2);
      const double dd = d11 + d2 * d2;
      if (dd < best) {
        best = dd;
        ba = a;
        bb = b;
      }
    }
  }
  const int k = gidx[(size_t)ba * n2 + bb];
  const cf* a = alpha + (size_t)v * r;
  const cf* d = dhr + (size_t)k * r;
  float nr = 0.f, ipr = 0.f, ipi = 0.f;
  for (int j = 0; j < r; ++j) {
    nr += a[j].x * a[j].x + a[j].y * a[j].y;
    ipr += d[j].x * a[j].x + d[j].y * a[j].y;
    ipi += d[j].x * a[j].y - d[j].y * a[j].x;
  }
  nr = sqrtf(nr);
  const float res = 1.f - sqrtf(ipr * ipr + ipi * ipi) / (nr > 0.f ? nr : 1.f);
  idx[v] = k;
  t12[(size_t)v * 2] = (float)exp(lt1);
  t12[(size_t)v * 2 + 1] = (float)exp(lt2);
  if (rho) rho[v] = fmaxf(ipr / norms[k], 0.f);
  if (resid) resid[v] = res;
  const int f = res > theta;
  fb[v] = f;
  if (f) fblist[atomicAdd(nfb, 1)] = v;
}

__global__ __launch_bounds__(256) void k_gather_alpha(const cf* __restrict__ alpha, const int* __restrict__ list,
                                                      const int* __restrict__ nfb, int r, cf* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nfb[0]) return;
  const int v = list[j];
  for (int k = 0; k < r; ++k) out[(size_t)j * r + k] = alpha[(size_t)v * r + k];
}

__global__ __launch_bounds__(256) void k_scatter_fb(const int* __restrict__ list, const int* __restrict__ nfb,
                                                    const int* __restrict__ fidx, const float* __restrict__ frho,
                                                    const float* __restrict__ lut, int nparam, int* __restrict__ idx,
                                                    float* __restrict__ t12, float* __restrict__ rho) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nfb[0]) return;
  const int v = list[j], k = fidx[j];
  idx[v] = k;
  t12[(size_t)v * 2] = lut[(size_t)k * nparam];
  t12[(size_t)v * 2 + 1] = lut[(size_t)k * nparam + 1];
  if (rho) rho[v] = frho[j];
}

__global__ void k_zero_int(int* p) { p[0] = 0; }

// ------------------------------------------------------------------ host side
template <bool BF16, int AL, int BL, int EPI>
mrf_status gemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc, const float* bias,
                const float* mask, int mld, int S, hipStream_t s, const char* name, float* asum = nullptr) {
  const int ks = (K + S - 1) / S;
  dim3 grid(ceil_div(N, kG), ceil_div(M, kG), S);
  if (BF16) {
    // float4 operand loads where the leading dimension, the rows and the k slices are multiples of
    // four (the column sums of A read the scalar tile)
    const bool a4 = !asum && lda % 4 == 0 && ((uintptr_t)A & 15) == 0 &&
                    (AL == LAY_K ? (K % 4 == 0 && ks % 4 == 0) : M % 4 == 0);
    const bool b4 = ldb % 4 == 0 && ((uintptr_t)B & 15) == 0 && (BL == LAY_K ? (K % 4 == 0 && ks % 4 == 0) : N % 4 == 0);
#define MRF_GB(A4, B4)                                                                                         \
  MRF_LAUNCH(name, s, k_gemm_bf16<AL, BL, EPI, A4, B4><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, \
                                                                           mask, mld, ks, asum))
    if (a4 && b4) MRF_GB(true, true);
    else if (b4) MRF_GB(false, true);
    else if (a4) MRF_GB(true, false);
    else MRF_GB(false, false);
#undef MRF_GB
  }
  else
    MRF_LAUNCH(name, s, k_gemm<false, AL, BL, EPI><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, mask, mld, ks));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// forward pass: acts[l] = [B][width_l]; acts[0] = z; returns y in acts[nl]
mrf_status mlp_forward(const mrf_mlp_s* P, bool bf16, int B, std::vector<float*>& acts, hipStream_t s) {
  mrf_status e;
  for (int l = 0; l < P->nl; ++l) {
    const float* W = P->p + P->offW[l];
    const float* b = P->p + P->offb[l];
    const bool last = l == P->nl - 1;
    const int in = P->lin[l], out = P->lout[l];
    if (bf16) {
      e = last ? gemm<true, LAY_K, LAY_K, EPI_BIAS>(B, out, in, acts[l], in, W, in, acts[l + 1], out, b, nullptr, 0, 1, s, "mlp_fwd")
               : gemm<true, LAY_K, LAY_K, EPI_BIAS_RELU>(B, out, in, acts[l], in, W, in, acts[l + 1], out, b, nullptr, 0, 1, s, "mlp_fwd");
    } else {
      e = last ? gemm<false, LAY_K, LAY_K, EPI_BIAS>(B, out, in, acts[l], in, W, in, acts[l + 1], out, b, nullptr, 0, 1, s, "mlp_fwd")
               : gemm<false, LAY_K, LAY_K, EPI_BIAS_RELU>(B, out, in, acts[l], in, W, in, acts[l + 1], out, b, nullptr, 0, 1, s, "mlp_fwd");
    }
    if (e) return e;
  }
  return MRF_OK;
}

struct TrainWs {
  float* z;                 // [B][nin]
  float* t;                 // [B][nout]
  std::vector<float*> acts; // nl + 1 activations (acts[0] = z)
  float *g0, *g1;           // [B][max width] gradient ping-pong
  float* part;              // split-K partials: BF16, layer l's [S][out in] and [S][out] at poff[l]
  std::vector<size_t> poff;
  float* lpart;             // loss partials
  float* loss;              // [1]
  unsigned* cnt;            // [1] the loss kernel's block counter (zeroed per call)
  size_t bytes;
};
constexpr int kSplitK = 16;
static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

TrainWs train_ws(const mrf_mlp_s* P, int B, void* base) {
  TrainWs w{};
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = p ? p + off : nullptr;
    off += al(b);
    return (float*)q;
  };
  const int wmax = std::max(P->hid, std::max(P->nin, P->nout));
  w.z = take((size_t)B * P->nin * 4);
  w.t = take((size_t)B * P->nout * 4);
  w.acts.push_back(w.z);
  for (int l = 0; l < P->nl; ++l) w.acts.push_back(take((size_t)B * P->lout[l] * 4));
  w.g0 = take((size_t)B * wmax * 4);
  w.g1 = take((size_t)B * wmax * 4);
  size_t np = 0;
  for (int l = 0; l < P->nl; ++l) {
    w.poff.push_back(np);
    np += (size_t)kSplitK * ((size_t)P->lout[l] * P->lin[l] + P->lout[l]);
  }
  w.part = take(std::max(np, (size_t)kSplitK * (wmax * wmax + wmax)) * 4);
  w.lpart = take((size_t)ceil_div((long)B * P->nout, 256) * 4);
  w.loss = take(4);
  w.cnt = (unsigned*)take(4);
  w.bytes = off;
  return w;
}

// the loss kernel's counter starts at zero in every call (the workspace is the caller's)
mrf_status zero_counters(const TrainWs& w, hipStream_t s) {
  MRF_LAUNCH("mlp_loss", s, k_zero_u32<<<1, 256, 0, s>>>(w.cnt, 1));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// loss and gradients of a batch (z, t already in the workspace, counter zero); grads into P->g
// and the loss into w.loss (and loss_out when set). BF16: the weight-gradient products leave
// their split-K slices per layer and one launch at the end sums them all, followed, with ad,
// by the Adam step (every backward product has read W by then); with next (rank r) that launch
// also writes the next training batch into the batch buffers.
mrf_status mlp_backward(mrf_mlp_s* P, bool bf16, int B, TrainWs& w, hipStream_t s, const AdamArgs* ad = nullptr,
                        float* loss_out = nullptr, const SynthArgs* next = nullptr, int r = 0) {
  mrf_status e;
  if ((e = mlp_forward(P, bf16, B, w.acts, s))) return e;
  const int n = B * P->nout;
  MRF_LAUNCH("mlp_loss", s, k_loss<<<ceil_div(n, 256), 256, 0, s>>>(w.acts[P->nl], w.t, n, 1.f / (float)n, w.g0,
                                                                    w.lpart, w.cnt, w.loss, loss_out));
  GradSegs sg{};
  int segmax = 0;
  float* gout = w.g0;   // dL/d(output of layer l), [B][lout[l]]
  float* gin = w.g1;
  for (int l = P->nl - 1; l >= 0; --l) {
    const int in = P->lin[l], out = P->lout[l];
    float* dW = P->g + P->offW[l];
    float* db = P->g + P->offb[l];
    const float* W = P->p + P->offW[l];
    // dW[out][in] = sum_b gout[b][out] h[b][in]: split over the batch, fixed-order reduction
    if (bf16) {
      // the BF16 product also sums gout's columns (the bias gradient, in FP32) per batch slice
      float* wpart = w.part + w.poff[l];
      float* dbpart = wpart + (size_t)kSplitK * out * in;
      // gin[b][in] = (sum_o gout[b][o] W[o][in]) * (h[b][in] > 0) in the same launch where the
      // operand layouts allow 16-byte loads of W and of h (as gemm() would choose them)
      const bool pair = l > 0 && in % 4 == 0 && ((uintptr_t)W & 15) == 0 && ((uintptr_t)w.acts[l] & 15) == 0;
      if (pair) {
        const bool da4 = out % 4 == 0 && ((uintptr_t)gout & 15) == 0;
        const int ksw = ceil_div(B, kSplitK);
        const GemmArgs d{B, in, out, gout, out, W, in, gin, in, w.acts[l], in, out, nullptr, ceil_div(in, kGB),
                         ceil_div(B, kGB)};
        const GemmArgs g{out, in, B, gout, out, w.acts[l], in, wpart, in, nullptr, 0, ksw, dbpart, ceil_div(in, kGB),
                         ceil_div(out, kGB)};
        const int nblk = d.gx * d.gy + g.gx * g.gy * kSplitK;
        if (da4) MRF_LAUNCH("mlp_bwd", s, k_gemm_bf16_bwd_pair<true><<<nblk, 256, 0, s>>>(d, g));
        else MRF_LAUNCH("mlp_bwd", s, k_gemm_bf16_bwd_pair<false><<<nblk, 256, 0, s>>>(d, g));
      } else {
        if (l > 0 && (e = gemm<true, LAY_K, LAY_MN, EPI_MASK>(B, in, out, gout, out, W, in, gin, in, nullptr, w.acts[l],
                                                               in, 1, s, "mlp_bwd")))
          return e;
        e = gemm<true, LAY_MN, LAY_MN, EPI_STORE>(out, in, B, gout, out, w.acts[l], in, wpart, in, nullptr, nullptr, 0,
                                                  kSplitK, s, "mlp_dw", dbpart);
        if (e) return e;
      }
      sg.part[sg.n] = wpart; sg.off[sg.n] = (long)P->offW[l]; sg.cnt[sg.n] = out * in; ++sg.n;
      sg.part[sg.n] = dbpart; sg.off[sg.n] = (long)P->offb[l]; sg.cnt[sg.n] = out; ++sg.n;
      segmax = std::max(segmax, out * in);
    } else {
      if (l > 0 && (e = gemm<false, LAY_K, LAY_MN, EPI_MASK>(B, in, out, gout, out, W, in, gin, in, nullptr, w.acts[l], in,
                                                              1, s, "mlp_bwd")))
        return e;
      e = gemm<false, LAY_MN, LAY_MN, EPI_STORE>(out, in, B, gout, out, w.acts[l], in, w.part, in, nullptr, nullptr, 0, kSplitK, s, "mlp_dw");
      if (e) return e;
      MRF_LAUNCH("mlp_dw_reduce", s, k_reduce_slices<<<ceil_div((long)out * in, 256), 256, 0, s>>>(w.part, kSplitK, (long)out * in, dW));
      // the split-K partials were consumed by the reduction above: their buffer holds these
      const int nch = ceil_div(B, kColRows);
      MRF_LAUNCH("mlp_db", s, k_colsum_part<<<dim3(ceil_div(out, 64), nch), 256, 0, s>>>(gout, B, out, w.part));
      MRF_LAUNCH("mlp_db", s, k_colsum_final<<<ceil_div(out, 256), 256, 0, s>>>(w.part, nch, out, db));
    }
    if (l > 0) std::swap(gout, gin);
  }
  if (bf16) {
    sg.gx = ceil_div(segmax, 256);
    const AdamArgs a = ad ? *ad : AdamArgs{};
    if (next)
      MRF_LAUNCH("mlp_grad_finish", s,
                 launch_finish_synth(r, sg.n * sg.gx + ceil_div(next->B, 256), s, sg, kSplitK, P->g, P->p, P->m, P->v, a,
                                     ad != nullptr, *next));
    else
      MRF_LAUNCH("mlp_grad_finish", s, k_grad_finish<<<sg.n * sg.gx, 256, 0, s>>>(sg, kSplitK, P->g, P->p, P->m, P->v, a,
                                                                                 ad != nullptr));
  }
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// the next Adam step's arguments (advances the step count)
AdamArgs adam_args(mrf_mlp_s* P, float lr, float b1, float b2, float eps) {
  P->t += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, P->t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, P->t)));
  return AdamArgs{lr, b1, b2, eps, c1, c2};
}

mrf_status adam(mrf_mlp_s* P, float lr, float b1, float b2, float eps, hipStream_t s) {
  const AdamArgs a = adam_args(P, lr, b1, b2, eps);
  MRF_LAUNCH("mlp_adam", s, k_adam<<<ceil_div((long)P->np, 256), 256, 0, s>>>(P->p, P->g, P->m, P->v, (long)P->np, a.lr,
                                                                             a.b1, a.b2, a.eps, a.c1, a.c2));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status ensure_stats(mrf_mlp_s* P, const mrf_dict_s* D, hipStream_t s) {
  if (P->have_stats) return MRF_OK;
  MRF_LAUNCH("mlp_stats", s, k_target_stats<<<1, 256, 0, s>>>(D->lut, D->M, D->nparam, P->stats));
  MRF_CHECK_LAUNCH();
  P->have_stats = true;
  return MRF_OK;
}

}  // namespace mrf

using namespace mrf;

extern "C" mrf_status mrf_mlp_create(int n_in, int hidden, int n_hidden_layers, int n_out, uint64_t seed, hipStream_t s,
                                     mrf_mlp_t* out) {
  clear_error();
  MRF_REQUIRE(out, MRF_INVALID_ARG, "mlp_create: null output");
  *out = nullptr;
  MRF_REQUIRE(n_in >= 1 && n_in <= 2 * kMaxR && hidden >= 1 && hidden <= 4096 && n_hidden_layers >= 1 &&
                  n_hidden_layers <= 8 && n_out == 2,
              MRF_INVALID_ARG, "mlp_create: need 1 <= n_in <= 32, 1 <= hidden <= 4096, 1..8 hidden layers, 2 outputs");
  auto* P = new mrf_mlp_s{};
  P->nin = n_in; P->hid = hidden; P->nhl = n_hidden_layers; P->nout = n_out; P->nl = n_hidden_layers + 1;
  size_t off = 0;
  for (int l = 0; l < P->nl; ++l) {
    const int in = l == 0 ? n_in : hidden, o = l == P->nl - 1 ? n_out : hidden;
    P->lin.push_back(in);
    P->lout.push_back(o);
    P->offW.push_back(off);
    off += (size_t)in * o;
    P->offb.push_back(off);
    off += o;
  }
  P->np = off;
  bool ok = hipMalloc(&P->p, off * 4) == hipSuccess && hipMalloc(&P->g, off * 4) == hipSuccess &&
            hipMalloc(&P->m, off * 4) == hipSuccess && hipMalloc(&P->v, off * 4) == hipSuccess &&
            hipMalloc(&P->stats, 4 * 8) == hipSuccess;
  if (!ok) {
    mrf_mlp_destroy(P);
    return fail(MRF_OOM, "mlp_create: device allocation failed");
  }
  hipError_t e = hipMemsetAsync(P->p, 0, off * 4, s);
  if (e == hipSuccess) e = hipMemsetAsync(P->m, 0, off * 4, s);
  if (e == hipSuccess) e = hipMemsetAsync(P->v, 0, off * 4, s);
  for (int l = 0; l < P->nl && e == hipSuccess; ++l) {
    const long n = (long)P->lin[l] * P->lout[l];
    k_init<<<ceil_div(n, 256), 256, 0, s>>>(P->p + P->offW[l], n, std::sqrt(2.f / P->lin[l]), (unsigned)l,
                                             (unsigned)seed, (unsigned)(seed >> 32));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    mrf_mlp_destroy(P);
    return fail(MRF_DEVICE, std::string("mlp_create: ") + hipGetErrorString(e));
  }
  *out = P;
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_destroy(mrf_mlp_t P) {
  clear_error();
  if (!P) return MRF_OK;
  hipFree(P->p); hipFree(P->g); hipFree(P->m); hipFree(P->v); hipFree(P->stats);
  hipFree(P->gidx); hipFree(P->i2max);
  delete P;
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_param_count(mrf_mlp_t P, size_t* n) {
  clear_error();
  MRF_REQUIRE(P && n, MRF_INVALID_ARG, "mlp_param_count: null argument");
  *n = P->np;
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_params(mrf_mlp_t P, float** params, float** grads) {
  clear_error();
  MRF_REQUIRE(P, MRF_INVALID_ARG, "mlp_params: null handle");
  if (params) *params = P->p;
  if (grads) *grads = P->g;
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_reset_optimizer(mrf_mlp_t P, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P, MRF_INVALID_ARG, "mlp_reset_optimizer: null handle");
  P->t = 0;
  MRF_CHECK_HIP(hipMemsetAsync(P->m, 0, P->np * 4, s));
  MRF_CHECK_HIP(hipMemsetAsync(P->v, 0, P->np * 4, s));
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_set_grid(mrf_mlp_t P, int n1, double log_t1_0, double dlog_t1, int n2, double log_t2_0,
                                       double dlog_t2, const int32_t* grid_index, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && grid_index && n1 >= 2 && n2 >= 2 && dlog_t1 > 0 && dlog_t2 > 0, MRF_INVALID_ARG,
              "mlp_set_grid: bad argument");
  std::vector<int> gi((size_t)n1 * n2), mx(n1, -1);
  MRF_CHECK_HIP(hipMemcpyAsync(gi.data(), grid_index, gi.size() * 4, hipMemcpyDeviceToHost, s));
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  int kmax = -1;
  for (int a = 0; a < n1; ++a)
    for (int b = 0; b < n2; ++b)
      if (gi[(size_t)a * n2 + b] >= 0) {
        mx[a] = b;
        kmax = std::max(kmax, (int)gi[(size_t)a * n2 + b]);
      }
  for (int a = 0; a < n1; ++a) {
    MRF_REQUIRE(mx[a] >= 0, MRF_INVALID_ARG, "mlp_set_grid: a T1 row without atoms");
    // the gate searches T2 indices 0 .. mx[a] of each row: they must all hold an atom
    for (int b = 0; b <= mx[a]; ++b)
      MRF_REQUIRE(gi[(size_t)a * n2 + b] >= 0, MRF_INVALID_ARG,
                  "mlp_set_grid: a row's kept T2 indices must run from 0 without gaps");
  }
  hipFree(P->gidx);
  hipFree(P->i2max);
  P->gidx = nullptr;
  P->i2max = nullptr;
  MRF_CHECK_HIP(hipMalloc(&P->gidx, gi.size() * 4));
  MRF_CHECK_HIP(hipMalloc(&P->i2max, (size_t)n1 * 4));
  MRF_CHECK_HIP(hipMemcpyAsync(P->gidx, gi.data(), gi.size() * 4, hipMemcpyHostToDevice, s));
  MRF_CHECK_HIP(hipMemcpyAsync(P->i2max, mx.data(), (size_t)n1 * 4, hipMemcpyHostToDevice, s));
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  P->n1 = n1; P->n2 = n2; P->l1_0 = log_t1_0; P->dl1 = dlog_t1; P->l2_0 = log_t2_0; P->dl2 = dlog_t2;
  P->gmax = kmax;
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_target_stats(mrf_mlp_t P, mrf_dict_t D, double* stats_host, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && D, MRF_INVALID_ARG, "mlp_target_stats: null handle");
  mrf_status e = ensure_stats(P, D, s);
  if (e) return e;
  if (stats_host) {
    MRF_CHECK_HIP(hipMemcpyAsync(stats_host, P->stats, 32, hipMemcpyDeviceToHost, s));
    MRF_CHECK_HIP(hipStreamSynchronize(s));
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_train_workspace_size(mrf_mlp_t P, int batch, size_t* bytes) {
  clear_error();
  MRF_REQUIRE(P && bytes && batch >= 1, MRF_INVALID_ARG, "mlp_train_workspace_size: bad argument");
  *bytes = train_ws(P, batch, nullptr).bytes;
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_synth(mrf_mlp_t P, mrf_dict_t D, uint64_t seed, int step, int batch, float snr_lo,
                                    float snr_hi, float* z, float* t, int32_t* m, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && D && z && t && batch >= 1 && step >= 0, MRF_INVALID_ARG, "mlp_synth: bad argument");
  MRF_REQUIRE(D->r >= 1 && 2 * D->r == P->nin, MRF_SHAPE, "mlp_synth: the dictionary needs a basis with 2 r = n_in");
  mrf_status e = ensure_stats(P, D, s);
  if (e) return e;
  const SynthArgs sa{D->dhr, D->M, D->lut, D->nparam, P->stats, (unsigned)seed, (unsigned)(seed >> 32), (unsigned)step,
                     batch, snr_lo, snr_hi, (float)D->L, z, t, m};
  MRF_LAUNCH("mlp_synth", s, launch_synth(D->r, dim3(ceil_div(batch, 256)), s, sa));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_forward(mrf_mlp_t P, const float* z, int batch, int bf16, float* y, void* ws,
                                      size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && z && y && batch >= 1, MRF_INVALID_ARG, "mlp_forward: bad argument");
  TrainWs w = train_ws(P, batch, ws);
  MRF_REQUIRE(ws && ws_bytes >= w.bytes, MRF_WORKSPACE, "mlp_forward: workspace too small");
  w.acts[0] = (float*)z;
  w.acts[P->nl] = y;
  return mlp_forward(P, bf16 != 0, batch, w.acts, s);
}

extern "C" mrf_status mrf_mlp_grads(mrf_mlp_t P, const float* z, const float* t, int batch, int bf16, float* loss,
                                    void* ws, size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && z && t && batch >= 1, MRF_INVALID_ARG, "mlp_grads: bad argument");
  TrainWs w = train_ws(P, batch, ws);
  MRF_REQUIRE(ws && ws_bytes >= w.bytes, MRF_WORKSPACE, "mlp_grads: workspace too small");
  MRF_CHECK_HIP(hipMemcpyAsync(w.z, z, (size_t)batch * P->nin * 4, hipMemcpyDeviceToDevice, s));
  MRF_CHECK_HIP(hipMemcpyAsync(w.t, t, (size_t)batch * P->nout * 4, hipMemcpyDeviceToDevice, s));
  mrf_status e = zero_counters(w, s);
  if (e) return e;
  return mlp_backward(P, bf16 != 0, batch, w, s, nullptr, loss);
}

extern "C" mrf_status mrf_mlp_adam_step(mrf_mlp_t P, float lr, float beta1, float beta2, float eps, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && lr >= 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f,
              MRF_INVALID_ARG, "mlp_adam_step: bad argument");
  return adam(P, lr, beta1, beta2, eps, s);
}

extern "C" mrf_status mrf_mlp_train(mrf_mlp_t P, mrf_dict_t D, const mrf_mlp_train_cfg* cfg, float* losses,
                                    void* ws, size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && D && cfg, MRF_INVALID_ARG, "mlp_train: null argument");
  MRF_REQUIRE(cfg->batch >= 1 && cfg->steps >= 0 && cfg->lr > 0.f && cfg->snr_hi >= cfg->snr_lo, MRF_INVALID_ARG,
              "mlp_train: bad configuration");
  MRF_REQUIRE(D->r >= 1 && 2 * D->r == P->nin, MRF_SHAPE, "mlp_train: the dictionary needs a basis with 2 r = n_in");
  TrainWs w = train_ws(P, cfg->batch, ws);
  MRF_REQUIRE(ws && ws_bytes >= w.bytes, MRF_WORKSPACE, "mlp_train: workspace too small");
  mrf_status e = ensure_stats(P, D, s);
  if (e) return e;
  if ((e = zero_counters(w, s))) return e;
  const int B = cfg->batch;
  const double pi = 3.14159265358979323846;
  auto batch_args = [&](int step) {
    return SynthArgs{D->dhr, D->M, D->lut, D->nparam, P->stats, (unsigned)cfg->seed, (unsigned)(cfg->seed >> 32),
                     (unsigned)step, B, cfg->snr_lo, cfg->snr_hi, (float)D->L, w.z, w.t, nullptr};
  };
  // BF16: each step's last launch also draws the next step's batch
  for (int it = 0; it < cfg->steps; ++it) {
    const int step = cfg->first_step + it;
    if (it == 0 || !cfg->bf16) MRF_LAUNCH("mlp_synth", s, launch_synth(D->r, dim3(ceil_div(B, 256)), s, batch_args(step)));
    const int T = cfg->total_steps > 0 ? cfg->total_steps : cfg->first_step + cfg->steps;
    const float lr = cfg->cosine ? (float)(cfg->lr * 0.5 * (1.0 + std::cos(pi * step / (double)T))) : cfg->lr;
    float* lo = losses ? losses + it : nullptr;
    if (cfg->bf16) {
      // the Adam step runs in the gradients' last launch
      const AdamArgs a = adam_args(P, lr, cfg->beta1, cfg->beta2, cfg->eps);
      const SynthArgs nx = batch_args(step + 1);
      if ((e = mlp_backward(P, true, B, w, s, &a, lo, it + 1 < cfg->steps ? &nx : nullptr, D->r))) return e;
    } else {
      if ((e = mlp_backward(P, false, B, w, s, nullptr, lo))) return e;
      if ((e = adam(P, lr, cfg->beta1, cfg->beta2, cfg->eps, s))) return e;
    }
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_match_workspace_size(mrf_mlp_t P, int Nv, size_t* bytes) {
  clear_error();
  MRF_REQUIRE(P && bytes && Nv >= 1, MRF_INVALID_ARG, "mlp_match_workspace_size: bad argument");
  *bytes = train_ws(P, Nv, nullptr).bytes + al((size_t)Nv * 4) * 4 + al((size_t)Nv * 2 * 4) + al(256) +
           al((size_t)Nv * kMaxR * sizeof(cf));
  return MRF_OK;
}

namespace mrf {
mrf_status match_subspace(const mrf_dict_s* D, const cf* alpha, int Nv, int* idx, float* rho, float* score,
                          float* params, hipStream_t s);
}

extern "C" mrf_status mrf_mlp_match(mrf_mlp_t P, mrf_dict_t D, const mrf_c64* alpha, int Nv, int bf16, float theta,
                                    int32_t* idx, float* t12, float* rho, float* resid, int32_t* fallback, int* n_fallback,
                                    void* ws, size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && D && alpha && idx && t12 && Nv >= 1, MRF_INVALID_ARG, "mlp_match: null argument");
  MRF_REQUIRE(P->gidx, MRF_INVALID_ARG, "mlp_match: call mrf_mlp_set_grid first");
  MRF_REQUIRE(P->gmax < D->M, MRF_SHAPE, "mlp_match: the gate's grid names atoms beyond the dictionary");
  MRF_REQUIRE(D->r >= 1 && 2 * D->r == P->nin, MRF_SHAPE, "mlp_match: the dictionary needs a basis with 2 r = n_in");
  size_t need = 0;
  mrf_mlp_match_workspace_size(P, Nv, &need);
  MRF_REQUIRE(ws && ws_bytes >= need, MRF_WORKSPACE, "mlp_match: workspace too small");
  mrf_status e = ensure_stats(P, D, s);
  if (e) return e;
  TrainWs w = train_ws(P, Nv, ws);
  char* base = (char*)ws + w.bytes;
  int* fb = fallback ? fallback : (int*)base;
  base += al((size_t)Nv * 4);
  int* list = (int*)base; base += al((size_t)Nv * 4);
  int* fidx = (int*)base; base += al((size_t)Nv * 4);
  float* frho = (float*)base; base += al((size_t)Nv * 4);
  float* yv = (float*)base; base += al((size_t)Nv * 2 * 4);
  int* nfb = (int*)base; base += al(256);
  cf* fa = (cf*)base;
  MRF_LAUNCH("mlp_features", s, k_features<<<ceil_div(Nv, 256), 256, 0, s>>>((const cf*)alpha, Nv, D->r, w.z));
  w.acts[P->nl] = yv;
  if ((e = mlp_forward(P, bf16 != 0, Nv, w.acts, s))) return e;
  MRF_LAUNCH("mlp_gate", s, k_zero_int<<<1, 1, 0, s>>>(nfb));
  MRF_LAUNCH("mlp_gate", s,
             k_gate<<<ceil_div(Nv, 256), 256, 0, s>>>(yv, P->stats, P->n1, P->n2, P->l1_0, P->dl1, P->l2_0, P->dl2, P->gidx,
                                                     P->i2max, D->dhr, D->norms, (const cf*)alpha, Nv, D->r, theta, idx, t12,
                                                     rho, resid, fb, nfb, list));
  MRF_CHECK_LAUNCH();
  int nf = 0;
  MRF_CHECK_HIP(hipMemcpyAsync(&nf, nfb, 4, hipMemcpyDeviceToHost, s));
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  if (n_fallback) *n_fallback = nf;
  if (nf > 0) {
    MRF_LAUNCH("mlp_fallback", s, k_gather_alpha<<<ceil_div(nf, 256), 256, 0, s>>>((const cf*)alpha, list, nfb, D->r, fa));
    if ((e = match_subspace(D, fa, nf, fidx, frho, nullptr, nullptr, s))) return e;
    MRF_LAUNCH("mlp_fallback", s,
               k_scatter_fb<<<ceil_div(nf, 256), 256, 0, s>>>(list, nfb, fidx, frho, D->lut, D->nparam, idx, t12, rho));
    MRF_CHECK_LAUNCH();
  }
  return MRF_OK;
}

// ------------------------------------------------------------------ save / load
namespace {
struct MlpHeader {
  uint64_t magic;
  int version, nin, hid, nhl, nout, t, have_stats, n1, n2, gmax, pad;
  uint64_t np;
  double l1_0, dl1, l2_0, dl2;
};
constexpr uint64_t kMlpMagic = 0x4d52464d4c507631ull;   // "MRFMLPv1"
size_t mal(size_t b) { return (b + 255) & ~(size_t)255; }
struct MlpLayout {
  size_t p, m, v, stats, gidx, i2max, total;
};
MlpLayout mlp_layout(const mrf_mlp_s* P) {
  MlpLayout c;
  c.p = mal(sizeof(MlpHeader));
  c.m = c.p + mal(P->np * 4);
  c.v = c.m + mal(P->np * 4);
  c.stats = c.v + mal(P->np * 4);
  c.gidx = c.stats + mal(32);
  c.i2max = c.gidx + mal((size_t)P->n1 * P->n2 * 4);
  c.total = c.i2max + mal((size_t)P->n1 * 4);
  return c;
}
}  // namespace

extern "C" mrf_status mrf_mlp_state_bytes(mrf_mlp_t P, size_t* bytes) {
  clear_error();
  MRF_REQUIRE(P && bytes, MRF_INVALID_ARG, "mlp_state_bytes: null argument");
  *bytes = mlp_layout(P).total;
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_save(mrf_mlp_t P, void* buf, size_t bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && buf, MRF_INVALID_ARG, "mlp_save: null argument");
  const MlpLayout c = mlp_layout(P);
  MRF_REQUIRE(bytes >= c.total, MRF_WORKSPACE, "mlp_save: buffer smaller than mrf_mlp_state_bytes");
  MlpHeader h{};
  h.magic = kMlpMagic;
  h.version = 1;
  h.nin = P->nin; h.hid = P->hid; h.nhl = P->nhl; h.nout = P->nout; h.t = P->t; h.have_stats = P->have_stats;
  h.n1 = P->gidx ? P->n1 : 0; h.n2 = P->gidx ? P->n2 : 0; h.gmax = P->gmax; h.np = P->np;
  h.l1_0 = P->l1_0; h.dl1 = P->dl1; h.l2_0 = P->l2_0; h.dl2 = P->dl2;
  char* o = (char*)buf;
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.p, P->p, P->np * 4, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.m, P->m, P->np * 4, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.v, P->v, P->np * 4, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.stats, P->stats, 32, hipMemcpyDefault, s));
  if (h.n1) {
    MRF_CHECK_HIP(hipMemcpyAsync(o + c.gidx, P->gidx, (size_t)h.n1 * h.n2 * 4, hipMemcpyDefault, s));
    MRF_CHECK_HIP(hipMemcpyAsync(o + c.i2max, P->i2max, (size_t)h.n1 * 4, hipMemcpyDefault, s));
  }
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  MRF_CHECK_HIP(hipMemcpy(o, &h, sizeof h, hipMemcpyDefault));
  return MRF_OK;
}

extern "C" mrf_status mrf_mlp_load(mrf_mlp_t P, const void* buf, size_t bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(P && buf, MRF_INVALID_ARG, "mlp_load: null argument");
  MlpHeader h{};
  const char* o = (const char*)buf;
  MRF_REQUIRE(bytes >= sizeof h, MRF_WORKSPACE, "mlp_load: buffer too small");
  MRF_CHECK_HIP(hipMemcpy(&h, o, sizeof h, hipMemcpyDefault));
  MRF_REQUIRE(h.magic == kMlpMagic && h.version == 1, MRF_INVALID_ARG, "mlp_load: not a saved MLP");
  MRF_REQUIRE(h.nin == P->nin && h.hid == P->hid && h.nhl == P->nhl && h.nout == P->nout && h.np == P->np, MRF_SHAPE,
              "mlp_load: the saved network's architecture differs from this one");
  // the layout with the saved grid's size
  const int n1 = P->n1, n2 = P->n2;
  P->n1 = h.n1;
  P->n2 = h.n2;
  const MlpLayout c = mlp_layout(P);
  P->n1 = n1;
  P->n2 = n2;
  MRF_REQUIRE(bytes >= c.total, MRF_WORKSPACE, "mlp_load: buffer smaller than the saved state");
  MRF_CHECK_HIP(hipMemcpyAsync(P->p, o + c.p, P->np * 4, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(P->m, o + c.m, P->np * 4, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(P->v, o + c.v, P->np * 4, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(P->stats, o + c.stats, 32, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  if (h.n1) {
    int *gi = nullptr, *mx = nullptr;
    if (hipMalloc(&gi, (size_t)h.n1 * h.n2 * 4) != hipSuccess || hipMalloc(&mx, (size_t)h.n1 * 4) != hipSuccess) {
      hipFree(gi);
      return fail(MRF_OOM, "mlp_load: device allocation failed");
    }
    MRF_CHECK_HIP(hipMemcpy(gi, o + c.gidx, (size_t)h.n1 * h.n2 * 4, hipMemcpyDefault));
    MRF_CHECK_HIP(hipMemcpy(mx, o + c.i2max, (size_t)h.n1 * 4, hipMemcpyDefault));
    hipFree(P->gidx);
    hipFree(P->i2max);
    P->gidx = gi;
    P->i2max = mx;
    P->n1 = h.n1; P->n2 = h.n2; P->gmax = h.gmax;
    P->l1_0 = h.l1_0; P->dl1 = h.dl1; P->l2_0 = h.l2_0; P->dl2 = h.dl2;
  }
  P->t = h.t;
  P->have_stats = h.have_stats != 0;
  return MRF_OK;
}
