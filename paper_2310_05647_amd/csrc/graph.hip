// Parameter-manifold patch graph and graph-Laplacian operators (Sec. III-A, eqs. (7)-(10), (15)).
//
//   w_ij = exp(-||Q_{q_i}(M) - Q_{q_j}(M)||^2 / sigma^2)      eq. (8)
//   L = D - W, D_ii = sum_j w_ij                              eq. (10)
//   S_L X = Q*(Q(X) L)                                        manifold gradient of eq. (15)
// The graph keeps, for every patch, its K nearest patches by squared feature distance (self
// excluded, ties to the lower index), symmetrised by W = max(W, W^T). Features are the p x p x 3
// patches of the (T1, T2, PD) maps, each channel divided by its maximum over the map. sigma^2 is
// the lower median of the positive directed K-NN squared distances unless given.
//
// Kernels: k_chan_max -> k_features -> k_knn_dist (distance tiles) -> k_knn_select (one wave per
// patch: bitwise search of the K-th distance, ordered ballot compaction) -> k_sigma (radix select
// of the median) -> dense symmetric W -> CSR rows with the diagonal D_ii (columns ascending) -> lmax = max_i D_ii.
// Laplacian apply: one block per s x s pixel cell and a chunk of frames; every pixel of a cell
// lies in the same patches, so the stencil (covering patch i, neighbour j, L_ij) is uniform
// across the block and each source pixel is the output pixel shifted by q_j - q_i.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "fft.hpp"
#include "patch.hpp"

struct mrf_graph_s {
  mrf::PatchGeom g;
  int kmax, K, nf;
  float* F;        // [Np][nf] features
  int* knn;        // [Np][kmax]
  float* knd2;     // [Np][kmax]
  float* W;        // [Np][Np]
  int* rowptr;     // [Np + 1]
  int* col;        // [cap]
  float* val;      // [cap]
  int* cnt;        // [Np]
  float* deg;      // [Np]
  float* mx;       // [3]
  double* scal;    // [4]: sigma2, lmax, nnz, positive distances
  double* part;    // [max quad-form blocks]
  size_t cap, npart;
  // the Laplacian trace on cells (p = 2 s; see k_qc_lists): per cell the merged (Delta, weight)
  // entries whose partner cell lies in the cell's LDS window, those outside it, and the diagonal
  // weight; built with the CSR
  bool qc;                // the geometry has the cell form
  int* qc_cnt;            // [2][nslot] entry counts (in window, outside)
  int* qc_ptr;            // [3][nslot + 1] exclusive scans of qc_cnt (the third is scratch)
  int2* qc_in;            // [2 cap] (packed Delta, weight bits)
  int2* qc_out;           // [2 cap]
  float* qc_wd;           // [nslot]
  int* qc_fslot;          // [nslot + 1]: slots with out-of-window entries, then their count
  int nslot, ntx;         // slots (tile-major cells, border tiles padded) and tiles per side
};

namespace mrf {


// Channel maxima of the (T1, T2, PD) maps in two steps: 64 blocks per channel reduce slices into
// pm[c][b], then one wave per channel takes the maximum of its 64 partials (1 if it is not
// positive). The maximum does not depend on the order of the comparisons.
constexpr int kCmBlocks = 64;
__global__ __launch_bounds__(256) void k_chan_max_part(const float* __restrict__ maps, int nn, float* __restrict__ pm) {
  __shared__ float red[4];
  const int c = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
  const int per = (nn + kCmBlocks - 1) / kCmBlocks, i0 = b * per, i1 = min(nn, i0 + per);
  float m = -3.4e38f;
  for (int i = i0 + t; i < i1; i += 256) m = fmaxf(m, maps[(size_t)c * nn + i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((t & 63) == 0) red[t >> 6] = m;
  __syncthreads();
  if (t == 0) pm[c * kCmBlocks + b] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}
__global__ __launch_bounds__(64 * 3) void k_chan_max_final(const float* __restrict__ pm, float* __restrict__ mx) {
  const int c = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float m = pm[c * kCmBlocks + lane];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) mx[c] = m > 0.f ? m : 1.f;
}

__global__ void k_features(const float* __restrict__ maps, const float* __restrict__ mx, PatchGeom g,
                           float* __restrict__ F) {
  const int pp = g.p * g.p, nf = 3 * pp;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)g.Np * nf) return;
  const int i = (int)(t / nf), f = (int)(t % nf);
  const int c = f / pp, r = f % pp;
  const int y = (i / g.n1) * g.s + r / g.p, x = (i % g.n1) * g.s + r % g.p;
  F[t] = maps[((size_t)c * g.N + y) * g.N + x] / mx[c];
}

// K-NN search in two kernels. k_knn_dist: squared feature distances of every patch pair, one
// 64 x 64 tile of pairs per block, only tiles on or above the diagonal; an off-diagonal tile is
// also stored transposed. Each pair sums fmaf(d, d, .) over the features in ascending order with
// d = F_i - F_j; (F_j - F_i)^2 is the same float, so the matrix is exactly symmetric and each
// distance has a single value wherever it is used. The matrix is written into the W buffer (it is
// cleared before W is filled). k_knn_select: one wave per patch; the row (self excluded) sits in
// registers, a bitwise search finds the K-th smallest distance, and an ordered ballot pass over
// the row takes every smaller one plus the lowest-index ties at that value, sorted by
// (distance, index).
constexpr int kKnnTile = 64;
constexpr int kKnnFch = 32;               // features per LDS chunk
constexpr int kKnnLd = kKnnTile + 4;      // LDS row stride (floats; keeps float4 rows aligned)

__global__ __launch_bounds__(256) void k_knn_dist(const float* __restrict__ F, int Np, int nf, int nt,
                                                  float* __restrict__ D) {
  __shared__ __align__(16) float sm[2 * kKnnFch * kKnnLd > kKnnTile * (kKnnTile + 1) ? 2 * kKnnFch * kKnnLd
                                                                                       : kKnnTile * (kKnnTile + 1)];
  float* Fa = sm;                         // [kKnnFch][kKnnLd], patches of the row tile
  float* Fb = sm + kKnnFch * kKnnLd;      // same for the column tile
  // upper-triangular tile (bi <= bj) from the linear block index
  int bi = 0, rem = blockIdx.x;
  while (rem >= nt - bi) {
    rem -= nt - bi;
    ++bi;
  }
  const int bj = bi + rem;
  const int i0 = bi * kKnnTile, j0 = bj * kKnnTile, t = threadIdx.x;
  const int ti = t & 15, tj = t >> 4;     // this thread: rows i0 + 4 ti + a, columns j0 + 4 tj + b
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int f0 = 0; f0 < nf; f0 += kKnnFch) {
    __syncthreads();
    for (int e = t; e < kKnnTile * kKnnFch; e += 256) {
      const int r = e / kKnnFch, c = e % kKnnFch, f = f0 + c;
      const int ia = i0 + r, jb = j0 + r;
      Fa[c * kKnnLd + r] = ia < Np && f < nf ? F[(size_t)ia * nf + f] : 0.f;
      Fb[c * kKnnLd + r] = jb < Np && f < nf ? F[(size_t)jb * nf + f] : 0.f;
    }
    __syncthreads();
    // zero-padded features beyond nf add fmaf(0, 0, acc) = acc
#pragma unroll 4
    for (int c = 0; c < kKnnFch; ++c) {
      const float4 x = *reinterpret_cast<const float4*>(Fa + c * kKnnLd + 4 * ti);
      const float4 y = *reinterpret_cast<const float4*>(Fb + c * kKnnLd + 4 * tj);
      const float xa[4] = {x.x, x.y, x.z, x.w}, yb[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const float d = xa[a] - yb[b];
          acc[a][b] = fmaf(d, d, acc[a][b]);
        }
    }
  }
  __syncthreads();
  float* T = sm;                          // [kKnnTile][kKnnTile + 1] staged output tile
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) T[(4 * ti + a) * (kKnnTile + 1) + 4 * tj + b] = acc[a][b];
  __syncthreads();
  const int lane = t & 63, w = t >> 6;
  for (int r = w; r < kKnnTile; r += 4) {
    const int i = i0 + r, j = j0 + lane;
    if (i < Np && j < Np) D[(size_t)i * Np + j] = T[r * (kKnnTile + 1) + lane];
  }
  if (bi != bj) {
    for (int r = w; r < kKnnTile; r += 4) {
      const int j = j0 + r, i = i0 + lane;
      if (i < Np && j < Np) D[(size_t)j * Np + i] = T[lane * (kKnnTile + 1) + r];
    }
  }
}

__device__ inline int wave_count(bool p) { return __popcll(__ballot(p)); }

// RC = values of the row per lane (Np <= 64 RC). Block: 4 waves, one row each.
template <int RC>
__global__ __launch_bounds__(256) void k_knn_select(const float* __restrict__ D, int Np, int K,
                                                    int* __restrict__ knn, float* __restrict__ knd2, int kmax) {
  __shared__ unsigned long long sel[4][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + w;
  const bool valid = i < Np;              // no early exit: the block meets at a barrier below
  const float* row = D + (size_t)(valid ? i : 0) * Np;
  unsigned u[RC];
#pragma unroll
  for (int c = 0; c < RC; ++c) {
    const int j = lane + 64 * c;
    // self and the padding past Np get the largest key; they are never among the K (K <= Np - 1)
    u[c] = valid && j < Np && j != i ? __float_as_uint(row[j]) : 0xffffffffu;
  }
  // v = the largest x with #{u < x} <= K - 1, i.e. the K-th smallest value (distances are
  // non-negative, so their bit patterns order like the values)
  unsigned v = 0u;
  for (int bit = 31; bit >= 0; --bit) {
    const unsigned cand = v | (1u << bit);
    int cnt = 0;
#pragma unroll
    for (int c = 0; c < RC; ++c) cnt += wave_count(u[c] < cand);
    if (cnt <= K - 1) v = cand;
  }
  int nless = 0;
#pragma unroll
  for (int c = 0; c < RC; ++c) nless += wave_count(u[c] < v);
  const int neq_take = K - nless;         // ties at v taken in index order
  const unsigned long long below = (1ull << lane) - 1ull;
  int taken = 0, eq_seen = 0;
#pragma unroll
  for (int c = 0; c < RC; ++c) {
    const int j = lane + 64 * c;
    const unsigned long long eqm = __ballot(u[c] == v && j < Np && j != i);
    const bool is_eq = (eqm >> lane) & 1ull;
    const bool take = u[c] < v || (is_eq && eq_seen + __popcll(eqm & below) < neq_take);
    const unsigned long long tm = __ballot(take);
    if (take && valid) sel[w][taken + __popcll(tm & below)] = ((unsigned long long)u[c] << 32) | (unsigned)j;
    taken += __popcll(tm);
    eq_seen += __popcll(eqm);
  }
  __syncthreads();
  if (valid && lane < K) {
    const unsigned long long key = sel[w][lane];
    int rank = 0;
    for (int k = 0; k < K; ++k) rank += sel[w][k] < key;
    knn[(size_t)i * kmax + rank] = (int)(key & 0xffffffffu);
    knd2[(size_t)i * kmax + rank] = __uint_as_float((unsigned)(key >> 32));
  }
}

// sigma^2: the lower median of the positive directed K-NN squared distances (1 if there are none).
// One block of 1024 threads; for Np K <= 65536 thread t holds values e = t + 1024 j in registers
// (at most 64 each), non-positive ones replaced by the largest key. The median's bit pattern (which
// orders like the value for non-negative floats) is then found bit by bit: the largest x with
// #{u < x} <= target, each count a block-wide sum.
__global__ __launch_bounds__(1024) void k_sigma(const float* __restrict__ knd2, int Np, int K, int kmax,
                                                float sigma2_user, double* __restrict__ scal) {
  constexpr int kPer = 64;
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int total = Np * K;
  unsigned u[kPer];
  int c = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int e = t + 1024 * j;
    const float v = e < total ? knd2[(size_t)(e / K) * kmax + e % K] : 0.f;
    const bool pos = v > 0.f;
    u[j] = pos ? __float_as_uint(v) : 0xffffffffu;
    c += pos;
  }
  auto block_sum = [&](int x) {   // every thread gets the block total
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    __syncthreads();
    if (lane == 0) wsum[w] = x;
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) tot += wsum[q];
    return tot;
  };
  const int npos = block_sum(c);
  if (sigma2_user > 0.f || npos == 0) {
    if (t == 0) {
      scal[0] = sigma2_user > 0.f ? (double)sigma2_user : 1.0;
      scal[3] = npos;
    }
    return;
  }
  const int target = (npos - 1) / 2;
  unsigned x = 0u;
  for (int bit = 31; bit >= 0; --bit) {
    const unsigned cand = x | (1u << bit);
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) cnt += u[j] < cand;
    if (block_sum(cnt) <= target) x = cand;
  }
  if (t == 0) {
    scal[0] = (double)__uint_as_float(x);
    scal[3] = npos;
  }
}

// The same by a 4-pass radix select from memory, for Np K > 65536.
__global__ __launch_bounds__(1024) void k_sigma_radix(const float* __restrict__ knd2, int Np, int K, int kmax,
                                                float sigma2_user, double* __restrict__ scal) {
  __shared__ int hist[256];
  __shared__ int cnt_s;
  __shared__ unsigned prefix_s;
  __shared__ int target_s;
  const int t = threadIdx.x;
  const int total = Np * K;
  if (t == 0) cnt_s = 0;
  __syncthreads();
  int c = 0;
  for (int e = t; e < total; e += 1024) c += knd2[(size_t)(e / K) * kmax + e % K] > 0.f;
  atomicAdd(&cnt_s, c);
  __syncthreads();
  const int npos = cnt_s;
  if (sigma2_user > 0.f || npos == 0) {
    if (t == 0) {
      scal[0] = sigma2_user > 0.f ? (double)sigma2_user : 1.0;
      scal[3] = npos;
    }
    return;
  }
  if (t == 0) {
    prefix_s = 0u;
    target_s = (npos - 1) / 2;
  }
  __syncthreads();
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    for (int b = t; b < 256; b += 1024) hist[b] = 0;
    __syncthreads();
    const unsigned prefix = prefix_s;
    const unsigned hmask = pass == 0 ? 0u : (0xffffffffu << (32 - 8 * pass));
    for (int e = t; e < total; e += 1024) {
      const float v = knd2[(size_t)(e / K) * kmax + e % K];
      if (!(v > 0.f)) continue;
      const unsigned u = __float_as_uint(v);
      if ((u & hmask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1);
    }
    __syncthreads();
    if (t == 0) {
      int tg = target_s, b = 0;
      while (tg >= hist[b]) {
        tg -= hist[b];
        ++b;
      }
      target_s = tg;
      prefix_s = prefix | ((unsigned)b << shift);
    }
    __syncthreads();
  }
  if (t == 0) {
    scal[0] = (double)__uint_as_float(prefix_s);
    scal[3] = npos;
  }
}

__global__ void k_fill_f(float* __restrict__ a, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_scatter_w(const int* __restrict__ knn, const float* __restrict__ knd2, int Np, int K, int kmax,
                            const double* __restrict__ scal, float* __restrict__ W) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)Np * K) return;
  const int i = (int)(t / K), k = (int)(t % K);
  const int j = knn[(size_t)i * kmax + k];
  const float w = expf(-knd2[(size_t)i * kmax + k] / (float)scal[0]);
  // when both (i, j) and (j, i) are K-NN edges the two writes carry the same value: the
  // distance is computed from the same features in the same order
  W[(size_t)i * Np + j] = w;
  W[(size_t)j * Np + i] = w;
}

// Per row: number of off-diagonal non-zeros (+1 for the diagonal) and the degree, summed in a
// fixed order (per-thread strided partial sums, then a tree).
__global__ __launch_bounds__(256) void k_row_stats(const float* __restrict__ W, int Np, int* __restrict__ cnt,
                                                   float* __restrict__ deg) {
  __shared__ float rs[256];
  __shared__ int rc[256];
  const int i = blockIdx.x, t = threadIdx.x;
  float s = 0.f;
  int c = 0;
  for (int j = t; j < Np; j += 256) {
    const float w = W[(size_t)i * Np + j];
    s += w;
    c += w != 0.f;
  }
  rs[t] = s;
  rc[t] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      rs[t] += rs[t + o];
      rc[t] += rc[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    deg[i] = rs[0];
    cnt[i] = rc[0] + 1;
  }
}

__global__ __launch_bounds__(1024) void k_scan_rowptr(const int* __restrict__ cnt, int Np, int* __restrict__ rowptr,
                                                      const float* __restrict__ deg, double* __restrict__ scal) {
  __shared__ int part[1024];
  __shared__ float mxs[1024];
  const int t = threadIdx.x;
  const int per = (Np + 1023) / 1024;
  int s = 0;
  float m = 0.f;
  for (int k = 0; k < per; ++k) {
    const int i = t * per + k;
    if (i < Np) {
      s += cnt[i];
      m = fmaxf(m, deg[i]);
    }
  }
  part[t] = s;
  mxs[t] = m;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan (Hillis-Steele)
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) mxs[t] = fmaxf(mxs[t], mxs[t + o]);
    __syncthreads();
  }
  int run = t == 0 ? 0 : part[t - 1];
  for (int k = 0; k < per; ++k) {
    const int i = t * per + k;
    if (i < Np) {
      rowptr[i] = run;
      run += cnt[i];
    }
  }
  if (t == 1023) {
    rowptr[Np] = part[1023];
    scal[1] = mxs[0];        // max(L) = largest degree
    scal[2] = part[1023];
  }
}

__global__ __launch_bounds__(256) void k_csr_fill(const float* __restrict__ W, const float* __restrict__ deg, int Np,
                                                  const int* __restrict__ rowptr, int* __restrict__ col,
                                                  float* __restrict__ val) {
  __shared__ int sc[256];
  const int i = blockIdx.x, t = threadIdx.x;
  int out = rowptr[i];
  for (int j0 = 0; j0 < Np; j0 += 256) {
    const int j = j0 + t;
    const float w = j < Np ? W[(size_t)i * Np + j] : 0.f;
    const int flag = j < Np && (w != 0.f || j == i);
    sc[t] = flag;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int v = t >= o ? sc[t - o] : 0;
      __syncthreads();
      sc[t] += v;
      __syncthreads();
    }
    if (flag) {
      const int pos = out + sc[t] - 1;
      col[pos] = j;
      val[pos] = j == i ? deg[i] : -w;
    }
    out += sc[255];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- Laplacian apply
constexpr int kLapFramesPerThread = 8;

// Y = Q*(Q(X) L) on full frames (QUAD = false), or the per-block partial sums of
// Re<X, Q*(Q(X) L)> (QUAD = true). Block: one cell, 256 threads = s^2 pixels x (256/s^2)
// frame lanes, each thread kLapFramesPerThread frames.
template <bool QUAD>
__global__ __launch_bounds__(256) void k_lap_full(const cf* __restrict__ X, cf* __restrict__ Y,
                                                  double* __restrict__ part, const int* __restrict__ rowptr,
                                                  const int* __restrict__ col, const float* __restrict__ val,
                                                  PatchGeom g, int L) {
  const int ss = g.s * g.s;
  const int nsub = 256 / ss;
  const int cell = blockIdx.x, t = threadIdx.x;
  const int cy = cell / g.nc, cx = cell % g.nc;
  const int pix = t % ss, fsub = t / ss;
  const int py = cy * g.s + pix / g.s, px = cx * g.s + pix % g.s;
  const int v = py * g.N + px;
  const int f0 = blockIdx.y * nsub * kLapFramesPerThread + fsub;
  const size_t NN = (size_t)g.N * g.N;
  cf acc[kLapFramesPerThread];
#pragma unroll
  for (int k = 0; k < kLapFramesPerThread; ++k) acc[k] = cf{0.f, 0.f};
  const bool active = t < nsub * ss;
  int alo, ahi, blo, bhi;
  cover_range(g, cy, alo, ahi);
  cover_range(g, cx, blo, bhi);
  for (int a = alo; a <= ahi; ++a) {
    for (int b = blo; b <= bhi; ++b) {
      const int i = a * g.n1 + b;
      const int e1 = rowptr[i + 1];
      for (int e = rowptr[i]; e < e1; ++e) {
        const int j = col[e];
        const float w = val[e];
        const int src = v + ((j / g.n1 - a) * g.N + (j % g.n1 - b)) * g.s;
#pragma unroll
        for (int k = 0; k < kLapFramesPerThread; ++k) {
          const int f = f0 + k * nsub;
          if (active && f < L) {
            const cf xv = X[(size_t)f * NN + src];
            acc[k].x += w * xv.x;
            acc[k].y += w * xv.y;
          }
        }
      }
    }
  }
  if (!QUAD) {
#pragma unroll
    for (int k = 0; k < kLapFramesPerThread; ++k) {
      const int f = f0 + k * nsub;
      if (active && f < L) Y[(size_t)f * NN + v] = acc[k];
    }
  } else {
    __shared__ double red[256];
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < kLapFramesPerThread; ++k) {
      const int f = f0 + k * nsub;
      if (active && f < L) {
        const cf xv = X[(size_t)f * NN + v];
        q += (double)xv.x * acc[k].x + (double)xv.y * acc[k].y;
      }
    }
    red[t] = q;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) red[t] += red[t + o];
      __syncthreads();
    }
    if (t == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
  }
}

// Tr(Q(X) L Q(X)^H) = sum_i L_ii ||q_i||^2 + 2 sum_{i<j} L_ij Re<q_i, q_j> (L symmetric), with
// q_i the patch i block of X over all frames. One wave per (patch i, chunk of 8 frames): lane =
// (pixel of the patch, frame lane), FPT frames each; the row's neighbours j > i are compacted
// into LDS (64 entries at a time), then streamed two at a time so that 2 FPT loads per lane are
// in flight.
// Blocks hold 8 patches of one chunk; XCD x takes the chunks c = x (mod 8), so each XCD's L2
// holds its 8 frames (4 MB at 256 x 256) while it runs over all patches.
__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
constexpr int kQuadFch64 = 8;             // frames per chunk for 8 x 8 patches
constexpr int kQuadFch16 = 8;             // and for 4 x 4 patches
// PV adjacent pixels per lane (PV = 2: one 16-byte load; needs an even stride and patch size)
template <int PV>
struct PixVec;
template <>
struct PixVec<1> {
  typedef cf T;
  __device__ static float dot(const T& a, const T& b) { return a.x * b.x + a.y * b.y; }
};
template <>
struct PixVec<2> {
  typedef float4 T;
  __device__ static float dot(const T& a, const T& b) { return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w; }
};
constexpr int kQuadWpb = 8;   // waves (patches) per block
template <int PP, int PV, int FCH>
__global__ __launch_bounds__(64 * kQuadWpb) void k_lap_quad_edges(const cf* __restrict__ X, const int* __restrict__ rowptr,
                                                        const int* __restrict__ col, const float* __restrict__ val,
                                                        PatchGeom g, int L, int nchunk, double* __restrict__ part) {
  typedef typename PixVec<PV>::T VT;
  constexpr int NPL = PP / PV;             // lanes per frame
  constexpr int NSUB = 64 / NPL;           // frame lanes per wave
  constexpr int FPT = FCH / NSUB;          // frames per lane
  static_assert(FPT >= 1, "chunk too small for the patch");
  __shared__ int sj[kQuadWpb][64];
  __shared__ float sw[kQuadWpb][64];
  const int b = blockIdx.x;
  const int q = b >> 3;
  const int ngrp = (g.Np + kQuadWpb - 1) / kQuadWpb;
  const int c = (q / ngrp) * 8 + (b & 7);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = (q % ngrp) * kQuadWpb + w;
  if (c >= nchunk || i >= g.Np) return;    // whole waves only; no block barrier below
  const int r = (lane % NPL) * PV, fsub = lane / NPL;
  const int off = (r / g.p) * g.N + r % g.p;
  const size_t NN = (size_t)g.N * g.N;
  const int oi = (i / g.n1) * g.s * g.N + (i % g.n1) * g.s;
  const int fbase = c * FCH + fsub;
  auto ld = [&](int f, int o) -> VT {
    VT v{};
    if (f < L) v = *reinterpret_cast<const VT*>(X + (size_t)f * NN + o);
    return v;
  };
  VT qi[FPT];
#pragma unroll
  for (int k = 0; k < FPT; ++k) qi[k] = ld(fbase + k * NSUB, oi + off);
  float s0 = 0.f;
#pragma unroll
  for (int k = 0; k < FPT; ++k) s0 += PixVec<PV>::dot(qi[k], qi[k]);
  double acc = 0.0;
  // sj holds each neighbour's patch origin offset (formed once per edge by the lane that read it)
  // the row in windows of 64 entries (a hub node's row can be longer than 2 K + 1)
  const int e0 = rowptr[i], e1 = rowptr[i + 1];
  for (int base = e0; base < e1; base += 64) {
    const bool has = base + lane < e1;
    const int cj = has ? col[base + lane] : -1;
    const float wj = has ? val[base + lane] : 0.f;
    const unsigned long long up = __ballot(cj > i);
    const unsigned long long dg = __ballot(cj == i);
    const int nup = __popcll(up);
    if (dg) acc += (double)__shfl(wj, __ffsll((long long)dg) - 1) * s0;
    if (cj > i) {
      const int pos = __popcll(up & ((1ull << lane) - 1ull));
      sj[w][pos] = (cj / g.n1) * g.s * g.N + (cj % g.n1) * g.s;
      sw[w][pos] = wj;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int m = 0;
    for (; m + 1 < nup; m += 2) {
      const int oa = sj[w][m] + off, ob = sj[w][m + 1] + off;
      VT xa[FPT], xb[FPT];
#pragma unroll
      for (int k = 0; k < FPT; ++k) {
        xa[k] = ld(fbase + k * NSUB, oa);
        xb[k] = ld(fbase + k * NSUB, ob);
      }
      float sa = 0.f, sb = 0.f;
#pragma unroll
      for (int k = 0; k < FPT; ++k) {
        sa += PixVec<PV>::dot(qi[k], xa[k]);
        sb += PixVec<PV>::dot(qi[k], xb[k]);
      }
      acc += 2.0 * ((double)sw[w][m] * sa + (double)sw[w][m + 1] * sb);
    }
    if (m < nup) {
      const int oa = sj[w][m] + off;
      float sa = 0.f;
#pragma unroll
      for (int k = 0; k < FPT; ++k) sa += PixVec<PV>::dot(qi[k], ld(fbase + k * NSUB, oa));
      acc += 2.0 * (double)sw[w][m] * sa;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();   // the window's list is read before the next one is written
  }
  acc = wave_sum_d(acc);
  if (lane == 0) part[(size_t)c * g.Np + i] = acc;
}

// ---------------------------------------------------------------- Laplacian trace on cells
// For p = 2 s every patch is 2 x 2 cells of s x s pixels, and cell (cy, cx) of patch i (origin
// cell (a, b)) is image cell (a + cy, b + cx). With Delta = origin(j) - origin(i) in cells,
//   Tr(Q L Q^H) = sum_cells c [ Wd(c) ||x_c||^2 + 2 sum_{Delta > 0} Wc(c, Delta) Re<x_c, x_{c+Delta}> ],
// Wd(c) = sum of L_ii over the patches i covering c, Wc(c, Delta) = sum of L_ij over the upper
// entries (j > i) of those rows with origin(j) - origin(i) = Delta; <x_c, x_d> runs over the s^2
// aligned pixels and all frames. Patches with similar neighbourhoods share (cell, Delta) pairs, so
// this touches each distinct pixel pair once instead of once per edge (2.7 times fewer at 256 x 256,
// K = 16). Cells are numbered tile-major ("slots": tile t of kQcTB x kQcTB cells, then the cell in
// the tile), so a tile's entries are one contiguous segment. The trace kernel stages a tile's
// window (the tile and a halo of kQcH cells) for kQcF frames at a time in LDS, with the tile's
// entries; pairs whose partner lies outside the window are summed by a second kernel that reads
// both cells from global memory.
// Launch shapes (measured choices; each may be set with -D when tuning)
#ifndef MRF_QC_TB
#define MRF_QC_TB 16
#endif
#ifndef MRF_QC_H
#define MRF_QC_H 4
#endif
#ifndef MRF_QC_F
#define MRF_QC_F 1
#endif
#ifndef MRF_QC_STAGES
#define MRF_QC_STAGES 16
#endif
#ifndef MRF_QC_WAVES
#define MRF_QC_WAVES 16
#endif
#ifndef MRF_QC_MINB
#define MRF_QC_MINB 1
#endif
#ifndef MRF_QC_FARBLOCKS
#define MRF_QC_FARBLOCKS 16384
#endif
constexpr int kQcTB = MRF_QC_TB, kQcH = MRF_QC_H, kQcF = MRF_QC_F;   // tile and halo (cells), frames per stage
constexpr int kQcStages = MRF_QC_STAGES;    // frame stages per trace block
constexpr int kQcWaves = MRF_QC_WAVES;      // waves per trace block
#ifndef MRF_QC_ECAP
#define MRF_QC_ECAP 3072
#endif
constexpr int kQcEcap = MRF_QC_ECAP;        // tile entries held in LDS (more are read from global memory)
constexpr int kQcRcap = 128;                // row entries staged in LDS by the list builder (a multiple of 64)
constexpr int kQcFarBlocks = MRF_QC_FARBLOCKS;

__device__ inline int qc_pack(int dy, int dx) { return (dy << 16) | (dx & 0xffff); }
__device__ inline int qc_dy(int k) { return k >> 16; }
__device__ inline int qc_dx(int k) { return (int)(short)(k & 0xffff); }

// slot -> cell coordinates (false for slots of border tiles that lie outside the image)
__device__ inline bool qc_slot_cell(int slot, int nc, int ntx, int& cy, int& cx) {
  const int tile = slot / (kQcTB * kQcTB), k = slot % (kQcTB * kQcTB);
  cy = (tile / ntx) * kQcTB + k / kQcTB;
  cx = (tile % ntx) * kQcTB + k % kQcTB;
  return cy < nc && cx < nc;
}

// Whether cell (qy, qx) lies in the trace window of the tile that holds cell (cy, cx).
__device__ inline bool qc_in_window(int cy, int cx, int qy, int qx) {
  const int ty0 = (cy / kQcTB) * kQcTB, tx0 = (cx / kQcTB) * kQcTB;
  return qy >= ty0 - kQcH && qy < ty0 + kQcTB + kQcH && qx >= tx0 - kQcH && qx < tx0 + kQcTB + kQcH;
}

// One wave per slot: the rows of the covering patches are staged in LDS with their merge keys
// (up to kQcRcap entries each, all loads in flight together; a longer row's tail is read from
// global memory), then lane 0 merges the off-diagonal entries of the four rows (columns ascending,
// so the key Delta = origin(j) - origin(i) ascends lexicographically within a row); equal Delta
// from several patches are summed in ascending patch order. A pair of cells {c, d = c + Delta}
// (Delta > 0 from c's upper entries, Delta < 0 from its lower ones) is summed once, by the side
// whose window holds the other cell: by c if d lies in c's window; otherwise by d if c lies in
// d's window (d then holds it as its entry -Delta); otherwise by the out-of-window kernel, listed
// under c. Each side decides from the same two window tests, and both sum the same L_ij in the
// same order, so every pair is taken exactly once. COUNT: entry counts (in window, outside) and the
// diagonal weight; otherwise the entries are written at the scanned offsets.
template <bool COUNT>
__global__ __launch_bounds__(256) void k_qc_lists(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                  const float* __restrict__ val, PatchGeom g, int ntx, int nslot,
                                                  int* __restrict__ cnt, const int* __restrict__ ptr,
                                                  int2* __restrict__ ent_in, int2* __restrict__ ent_out,
                                                  float* __restrict__ wd, size_t cap2) {
  constexpr int RPL = kQcRcap / 64;   // staged entries per lane and row
  __shared__ int skey[4][4][kQcRcap];
  __shared__ float sval[4][4][kQcRcap];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = blockIdx.x * 4 + w;
  if (slot >= nslot) return;                  // whole waves; no block barrier below
  int cy, cx;
  const bool live = qc_slot_cell(slot, g.nc, ntx, cy, cx);
  const int M = 2 * g.n1;   // key = dy M + dx orders Delta lexicographically (|dx| < n1); 0 = diagonal
  int pi[4], r0[4], r1[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int ay = cy - 1 + (k >> 1), bx = cx - 1 + (k & 1);
    const bool on = live && ay >= 0 && bx >= 0 && ay < g.n1 && bx < g.n1;
    pi[k] = on ? ay * g.n1 + bx : -1;
    r0[k] = on ? rowptr[pi[k]] : 0;
    r1[k] = on ? rowptr[pi[k] + 1] : 0;
  }
  int cv[4][RPL];
  float vv[4][RPL];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int e = r0[k] + lane + 64 * r;
      const bool in = e < r1[k];
      cv[k][r] = in ? col[e] : -1;
      vv[k][r] = in ? val[e] : 0.f;
    }
  float dg[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float d = 0.f;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int j = cv[k][r];
      const int key = j >= 0 ? (j / g.n1 - pi[k] / g.n1) * M + (j % g.n1 - pi[k] % g.n1) : 0x7fffffff;
      skey[w][k][lane + 64 * r] = key;
      sval[w][k][lane + 64 * r] = vv[k][r];
      d += key == 0 ? vv[k][r] : 0.f;   // the diagonal (one lane of the row at most)
    }
    // the row's diagonal, whichever lane holds it (zero when it lies beyond the staged part)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
    dg[k] = d;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane != 0) return;
  if (COUNT)
    for (int k = 0; k < 4; ++k)   // a diagonal beyond the staged part of a long row
      if (pi[k] >= 0 && r1[k] - r0[k] > kQcRcap && dg[k] == 0.f) {
        int lo = r0[k] + kQcRcap, hi = r1[k];
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (col[mid] < pi[k]) lo = mid + 1;
          else hi = mid;
        }
        if (lo < r1[k] && col[lo] == pi[k]) dg[k] = val[lo];
      }
  int pos[4], end[4];
  for (int k = 0; k < 4; ++k) {
    pos[k] = 0;
    end[k] = r1[k] - r0[k];
  }
  auto keyat = [&](int k) {
    if (pos[k] < kQcRcap) return skey[w][k][pos[k]];
    const int j = col[r0[k] + pos[k]];
    return (j / g.n1 - pi[k] / g.n1) * M + (j % g.n1 - pi[k] % g.n1);
  };
  auto valat = [&](int k) { return pos[k] < kQcRcap ? sval[w][k][pos[k]] : val[r0[k] + pos[k]]; };
  int nin = 0, nout = 0;
  const int base_in = COUNT ? 0 : ptr[slot], base_out = COUNT ? 0 : ptr[nslot + 1 + slot];
  while (true) {
    int best = 0x7fffffff;
    int keys[4];
    for (int k = 0; k < 4; ++k) {
      keys[k] = pi[k] >= 0 && pos[k] < end[k] ? keyat(k) : 0x7fffffff;
      best = min(best, keys[k]);
    }
    if (best == 0x7fffffff) break;
    float wsum = 0.f;
    for (int k = 0; k < 4; ++k)
      if (keys[k] == best) {
        wsum += valat(k);
        ++pos[k];
      }
    if (best == 0) continue;                  // the diagonal: Wd
    const int dy = (best + g.n1 + M * g.n1) / M - g.n1, dx = best - dy * M;
    const int ny = cy + dy, nx = cx + dx;
    const bool mine = qc_in_window(cy, cx, ny, nx);        // the partner lies in this cell's window
    const bool theirs = qc_in_window(ny, nx, cy, cx);      // this cell lies in the partner's window
    int where;                                 // 0: in-window list, 1: out-of-window list, -1: not here
    if (best > 0) where = mine ? 0 : (theirs ? -1 : 1);
    else where = (!theirs && mine) ? 0 : -1;  // the partner owns the pair (upper side)
    if (where < 0) continue;
    if (!COUNT) {
      // in-window entries carry the partner's offset in the trace kernel's LDS window (rows of
      // (kQcTB + 2 kQcH) s + 2 pixels), out-of-window ones its offset in the image
      const int wstr = (kQcTB + 2 * kQcH) * g.s + 2;
      const int off = where == 0 ? (dy * wstr + dx) * g.s : (dy * g.N + dx) * g.s;
      const int2 e = make_int2(off, __float_as_int(wsum));
      if (where == 0) {
        if ((size_t)(base_in + nin) < cap2) ent_in[base_in + nin] = e;
      } else if ((size_t)(base_out + nout) < cap2) {
        ent_out[base_out + nout] = e;
      }
    }
    if (where == 0) ++nin;
    else ++nout;
  }
  if (COUNT) {
    cnt[slot] = nin;
    cnt[nslot + slot] = nout;
    wd[slot] = (dg[0] + dg[1]) + (dg[2] + dg[3]);
  }
}

// One block: exclusive scans of the two count arrays [2][n] into ptr [2][n + 1], and the list of
// slots with out-of-window entries (fslot, its length in *nfs).
__global__ __launch_bounds__(1024) void k_qc_scan(const int* __restrict__ cnt, int n, int* __restrict__ ptr,
                                                  int* __restrict__ fslot, int* __restrict__ nfs) {
  __shared__ int part[1024];
  const int t = threadIdx.x, per = (n + 1023) / 1024;
  for (int h = 0; h < 3; ++h) {
    const int* cc = cnt + (size_t)(h == 0 ? 0 : n);
    int* pp = ptr + (size_t)h * (n + 1);
    int sum = 0;
    for (int k = 0; k < per; ++k) {
      const int i = t * per + k;
      if (i < n) sum += h < 2 ? cc[i] : (cc[i] > 0);
    }
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int v = t >= o ? part[t - o] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int run = t == 0 ? 0 : part[t - 1];
    for (int k = 0; k < per; ++k) {
      const int i = t * per + k;
      if (i < n) {
        if (h < 2) {
          pp[i] = run;
          run += cc[i];
        } else if (cc[i] > 0) {
          fslot[run++] = i;
        }
      }
    }
    if (t == 1023) {
      if (h < 2) pp[n] = part[1023];
      else nfs[0] = part[1023];
    }
    __syncthreads();
  }
}

// Trace over in-window pairs. Block: one tile of kQcTB^2 cells and kQcStages x kQcF frames; the
// tile's entries (up to kQcEcap) and, stage by stage, the window (tile + halo) of kQcF frames are
// held in LDS (rows padded by S pixels so that the S rows of a cell fall in different banks).
// Lanes: S rows x (64 / S) cells; each lane keeps its row of its cell and runs over the cell's
// entries (a wave holds one row of 16 cells of the tile when S = 4). Blocks are dealt to XCDs by
// frame chunk (chunk c on XCD c mod 8), so the tiles of a chunk share an L2.
template <int S>
__global__ __launch_bounds__(64 * kQcWaves, MRF_QC_MINB) void k_qc_trace(const cf* __restrict__ X,
                                                     const int* __restrict__ ptr,
                                                     const int2* __restrict__ ent, const float* __restrict__ wd,
                                                     PatchGeom g, int L, int ntx, int nfc, double* __restrict__ part) {
  constexpr int NTHR = 64 * kQcWaves;
  constexpr int WPX = (kQcTB + 2 * kQcH) * S;
  // window row stride (pixels): a row is 2 (mod 8) 16-byte units longer than a multiple of 128
  // bytes, so the 8 lanes of an LDS pass (4 cells x 2 rows, below) read 8 different bank groups
  constexpr int STR = WPX + 2;
  constexpr int NT = kQcTB * kQcTB;
  constexpr int CPW = 64 / S;                             // cells per wave: one lane per cell row
  constexpr int WPF = kQcWaves / kQcF;                    // waves per frame of a stage
  static_assert(kQcWaves % kQcF == 0, "the waves split evenly over a stage's frames");
  constexpr int STEPS = (NT + WPF * CPW - 1) / (WPF * CPW);
  typedef typename PixVec<2>::T VT;                       // two pixels (16 bytes)
  __shared__ __align__(16) cf win[kQcF][WPX][STR];
  __shared__ int2 sent[kQcEcap];
  __shared__ int lp[NT + 1];
  __shared__ float swd[NT];
  __shared__ double red[kQcWaves];
  const int b = blockIdx.x;
  const int ntile = ntx * ntx;
  const int q = b >> 3;
  const int tile = q % ntile;
  const int fc = (q / ntile) * 8 + (b & 7);
  if (fc >= nfc) {                                        // whole block, before any barrier
    if (threadIdx.x == 0) part[b] = 0.0;                  // the sum covers every block's partial
    return;
  }
  const int ty = tile / ntx, tx = tile % ntx;
  const int wy0 = (ty * kQcTB - kQcH) * S, wx0 = (tx * kQcTB - kQcH) * S;
  const int tp0 = ptr[tile * NT];
  const int nent = ptr[tile * NT + NT] - tp0;
  for (int t = threadIdx.x; t <= NT; t += NTHR) lp[t] = ptr[tile * NT + t] - tp0;
  for (int t = threadIdx.x; t < NT; t += NTHR) swd[t] = wd[tile * NT + t];
  for (int t = threadIdx.x; t < min(nent, kQcEcap); t += NTHR) sent[t] = ent[tp0 + t];
  const size_t NN = (size_t)g.N * g.N;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int fsel = w / WPF, wf = w % WPF;                 // this wave's frame of the stage, and its rank there
  // lane -> (cell of the wave, row of the cell): lanes 4m .. 4m + 3 hold four neighbouring cells
  const int uy = (lane >> 2) % S, lc = (lane & 3) + 4 * (lane / (4 * S));
  // window staging: float4 = two pixels (window columns start at even pixels: S even, N even).
  // The loads of stage k + 1 are issued before the compute of stage k, so they are in flight
  // while it runs.
  constexpr int Q4 = WPX / 2;
  constexpr int NTOT = kQcF * WPX * Q4;
  constexpr int NLD = (NTOT + NTHR - 1) / NTHR;
  const int nstage = min(kQcStages, (L - fc * kQcStages * kQcF + kQcF - 1) / kQcF);
  // this thread's part of the window: frame, pixel offset in the frame (-1 outside the image) and
  // LDS position of each of its NLD pixel pairs, the same for every stage
  int gofs[NLD], lofs[NLD], fof[NLD];
#pragma unroll
  for (int r = 0; r < NLD; ++r) {
    const int t = threadIdx.x + r * NTHR;
    const int f = t / (WPX * Q4), rem = t % (WPX * Q4);
    const int y = rem / Q4, x2 = (rem % Q4) * 2;
    const int gy = wy0 + y, gx = wx0 + x2;
    fof[r] = f;
    gofs[r] = t < NTOT && gy >= 0 && gy < g.N && gx >= 0 && gx < g.N ? gy * g.N + gx : -1;
    lofs[r] = (f * WPX + y) * STR + x2;
  }
  float4 v[NLD];
  auto issue = [&](int stg) {
    const int f0 = (fc * kQcStages + stg) * kQcF;
    const cf* xf = X + (size_t)f0 * NN;
#pragma unroll
    for (int r = 0; r < NLD; ++r)
      v[r] = gofs[r] >= 0 && f0 + fof[r] < L ? *reinterpret_cast<const float4*>(xf + (size_t)fof[r] * NN + gofs[r])
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  issue(0);
  double acc = 0.0;
  for (int stg = 0; stg < nstage; ++stg) {
    const int f0 = (fc * kQcStages + stg) * kQcF;
    __syncthreads();                                      // the previous stage's window is read
#pragma unroll
    for (int r = 0; r < NLD; ++r)
      if (gofs[r] >= 0 && f0 + fof[r] < L) *reinterpret_cast<float4*>(&win[0][0][0] + lofs[r]) = v[r];
    __syncthreads();
    if (stg + 1 < nstage) issue(stg + 1);
    // frames past L were not staged: their waves skip them, never multiplying by zero
    if (f0 + fsel >= L) continue;
    const cf* wbase = &win[fsel][0][0];
    for (int st = 0; st < STEPS; ++st) {
      const int k = (wf * STEPS + st) * CPW + lc;         // cell in the tile
      const int tcy = k / kQcTB, tcx = k % kQcTB;
      if (k >= NT || ty * kQcTB + tcy >= g.nc || tx * kQcTB + tcx >= g.nc) continue;
      const int base = ((tcy + kQcH) * S + uy) * STR + (tcx + kQcH) * S;   // this lane's cell row
      VT xa[S / 2];
      float d = 0.f;
#pragma unroll
      for (int h = 0; h < S / 2; ++h) {
        xa[h] = *reinterpret_cast<const VT*>(wbase + base + 2 * h);
        d += PixVec<2>::dot(xa[h], xa[h]);
      }
      float off = 0.f;
      const int e1 = lp[k + 1];
      int e = lp[k];
      // two entries per step: their window reads are in flight together
      for (; e + 1 < e1; e += 2) {
        const int2 ea = e < kQcEcap ? sent[e] : ent[tp0 + e];
        const int2 eb = e + 1 < kQcEcap ? sent[e + 1] : ent[tp0 + e + 1];
        float da = 0.f, db = 0.f;
#pragma unroll
        for (int h = 0; h < S / 2; ++h) {
          const VT va = *reinterpret_cast<const VT*>(wbase + base + ea.x + 2 * h);
          const VT vb = *reinterpret_cast<const VT*>(wbase + base + eb.x + 2 * h);
          da += PixVec<2>::dot(xa[h], va);
          db += PixVec<2>::dot(xa[h], vb);
        }
        off += __int_as_float(ea.y) * da;
        off += __int_as_float(eb.y) * db;
      }
      if (e < e1) {
        const int2 en = e < kQcEcap ? sent[e] : ent[tp0 + e];
        float dot = 0.f;
#pragma unroll
        for (int h = 0; h < S / 2; ++h)
          dot += PixVec<2>::dot(xa[h], *reinterpret_cast<const VT*>(wbase + base + en.x + 2 * h));
        off += __int_as_float(en.y) * dot;
      }
      acc += (double)swd[k] * (double)d + 2.0 * (double)off;
    }
  }
  acc = wave_sum_d(acc);
  if (lane == 0) red[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kQcWaves; ++k) t += red[k];
    part[b] = t;
  }
}

// Trace over the out-of-window pairs. Work items are (slot with such entries, chunk of
// 128 / S^2 frames); XCD x (blocks b = x mod 8) takes the chunks c = x (mod 8), and its waves run
// through all slots of one chunk before the next, so the frames in use fit the XCD's L2. Each
// wave sums its items into one partial. Lanes: the S rows x S/2 pixel pairs of the cell x the
// chunk's frames; a wave reads a batch of 64 entries with one load per lane and hands them round
// by lane exchange.
template <int S>
__global__ __launch_bounds__(256) void k_qc_far(const cf* __restrict__ X, const int* __restrict__ ptr,
                                                const int2* __restrict__ ent, const int* __restrict__ fslot,
                                                const int* __restrict__ nfs, PatchGeom g, int L, int ntx,
                                                double* __restrict__ part) {
  typedef typename PixVec<2>::T VT;
  constexpr int PPL = S * (S / 2);                        // pixel pairs of a cell
  constexpr int FCH = 64 / PPL;                           // frames per chunk
  const int lane = threadIdx.x & 63;
  const int xcd = blockIdx.x & 7;
  const int wl = (blockIdx.x >> 3) * 4 + (threadIdx.x >> 6);   // wave rank within its XCD
  const int nwl = (gridDim.x >> 3) * 4;
  const int nf = nfs[0];
  const int nchunk = (L + FCH - 1) / FCH;
  const int nchx = (nchunk - xcd + 7) / 8;                // chunks of this XCD
  const int nitem = nf * nchx;
  const int pp = lane % PPL, fl = lane / PPL;
  const int uy = pp / (S / 2), h = pp % (S / 2);
  const size_t NN = (size_t)g.N * g.N;
  double acc = 0.0;
  for (int it = wl; it < nitem; it += nwl) {
    const int cq = it / nf, slot = fslot[it - cq * nf];
    const int f = (xcd + 8 * cq) * FCH + fl;
    int cy, cx;
    qc_slot_cell(slot, g.nc, ntx, cy, cx);
    const int pa = (cy * S + uy) * g.N + cx * S + 2 * h;   // this lane's pixel pair
    const bool fv = f < L;
    const VT xa = fv ? *reinterpret_cast<const VT*>(X + (size_t)f * NN + pa) : VT{};
    float off = 0.f;
    const int e0 = ptr[slot], e1 = ptr[slot + 1];
    for (int eb = e0; eb < e1; eb += 64) {
      const int2 mine = eb + lane < e1 ? ent[eb + lane] : make_int2(0, 0);
      const int n = min(64, e1 - eb);
      int m = 0;
      for (; m + 1 < n; m += 2) {                         // two entries' loads in flight
        const int pa_ = __shfl(mine.x, m), wa = __shfl(mine.y, m);
        const int pb_ = __shfl(mine.x, m + 1), wb = __shfl(mine.y, m + 1);
        if (fv) {
          const VT va = *reinterpret_cast<const VT*>(X + (size_t)f * NN + pa + pa_);
          const VT vb = *reinterpret_cast<const VT*>(X + (size_t)f * NN + pa + pb_);
          off += __int_as_float(wa) * PixVec<2>::dot(xa, va);
          off += __int_as_float(wb) * PixVec<2>::dot(xa, vb);
        }
      }
      if (m < n) {
        const int po = __shfl(mine.x, m), wv = __shfl(mine.y, m);
        if (fv) off += __int_as_float(wv) * PixVec<2>::dot(xa, *reinterpret_cast<const VT*>(X + (size_t)f * NN + pa + po));
      }
    }
    acc += 2.0 * (double)off;
  }
  acc = wave_sum_d(acc);
  if (lane == 0) part[(size_t)xcd * nwl + wl] = acc;
}

// S_L applied to per-voxel subspace coefficients A[v][k] (k < r), voxel-major. Four threads per
// voxel: thread q of a quad takes the covering patches q, q + 4, ... of the voxel's cell (in
// raster order of (a, b)) and sums their rows of L; the quad's partial sums then meet by two
// quad exchanges in a fixed order. For even r each neighbour's coefficients are read as 16-byte
// pairs.
__device__ inline float quad_xor_add(float x, int ctrl_xor1) {
  return x + __int_as_float(ctrl_xor1 ? __builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false)
                                      : __builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, false));
}
__global__ __launch_bounds__(256) void k_lap_sub(const cf* __restrict__ A, cf* __restrict__ Y,
                                                 const int* __restrict__ rowptr, const int* __restrict__ col,
                                                 const float* __restrict__ val, PatchGeom g, int r) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const int v = (int)(t >> 2), q = (int)(t & 3);
  const bool live = v < g.N * g.N;   // no early exit: the quad exchanges need all four lanes
  cf acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = cf{0.f, 0.f};
  if (live) {
    const int py = v / g.N, px = v % g.N;
    const int cy = py / g.s, cx = px / g.s;
    int alo, ahi, blo, bhi;
    cover_range(g, cy, alo, ahi);
    cover_range(g, cx, blo, bhi);
    const int nb = bhi - blo + 1, ncov = (ahi - alo + 1) * nb;
    for (int c = q; c < ncov; c += 4) {
      const int a = alo + c / nb, b = blo + c % nb;
      const int i = a * g.n1 + b;
      for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int j = col[e];
        const float w = val[e];
        const int src = v + ((j / g.n1 - a) * g.N + (j % g.n1 - b)) * g.s;
        if ((r & 1) == 0) {
          const float4* Ap = reinterpret_cast<const float4*>(A + (size_t)src * r);
#pragma unroll
          for (int k2 = 0; k2 < 8; ++k2)
            if (2 * k2 < r) {
              const float4 av = Ap[k2];
              acc[2 * k2].x += w * av.x;
              acc[2 * k2].y += w * av.y;
              acc[2 * k2 + 1].x += w * av.z;
              acc[2 * k2 + 1].y += w * av.w;
            }
        } else {
#pragma unroll
          for (int k = 0; k < 16; ++k)
            if (k < r) {
              const cf av = A[(size_t)src * r + k];
              acc[k].x += w * av.x;
              acc[k].y += w * av.y;
            }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < r) {
      acc[k].x = quad_xor_add(quad_xor_add(acc[k].x, 1), 0);
      acc[k].y = quad_xor_add(quad_xor_add(acc[k].y, 1), 0);
    }
  if (live && q == 0) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < r) Y[(size_t)v * r + k] = acc[k];
  }
}

// First stage of a deterministic sum: block b adds the contiguous range [b*per, (b+1)*per).
__global__ __launch_bounds__(256) void k_sum_stage(const double* __restrict__ part, long n, long per,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  const long lo = (long)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  double s = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Deterministic sum of block partials (single block, fixed order) into out[0].
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, long n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// -------------------------------------------------------------- internal entry points
mrf_status sum_partials2(const double* part, long n, double* tmp, double* out, hipStream_t s);

// Cell entry lists of the Laplacian trace from the current CSR (p = 2 s only).
mrf_status qc_build(mrf_graph_s* G, hipStream_t s) {
  if (!G->qc) return MRF_OK;
  const PatchGeom& g = G->g;
  const int n = G->nslot;
  const size_t cap2 = 2 * G->cap;
  int* nfs = G->qc_fslot + n;
  MRF_LAUNCH("graph_qc_lists", s,
             k_qc_lists<true><<<ceil_div(n, 4), 256, 0, s>>>(G->rowptr, G->col, G->val, g, G->ntx, n, G->qc_cnt, nullptr,
                                                            nullptr, nullptr, G->qc_wd, cap2));
  MRF_LAUNCH("graph_qc_lists", s, k_qc_scan<<<1, 1024, 0, s>>>(G->qc_cnt, n, G->qc_ptr, G->qc_fslot, nfs));
  MRF_LAUNCH("graph_qc_lists", s,
             k_qc_lists<false><<<ceil_div(n, 4), 256, 0, s>>>(G->rowptr, G->col, G->val, g, G->ntx, n, nullptr,
                                                             G->qc_ptr, G->qc_in, G->qc_out, nullptr, cap2));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status graph_build(mrf_graph_s* G, const float* maps, int K, float sigma2, hipStream_t s) {
  const PatchGeom& g = G->g;
  const int nf = 3 * g.p * g.p;
  float* pm = reinterpret_cast<float*>(G->part);   // 3 x kCmBlocks partial maxima (the buffer is free here)
  MRF_LAUNCH("graph_chan_max", s, k_chan_max_part<<<dim3(kCmBlocks, 3), 256, 0, s>>>(maps, g.N * g.N, pm));
  MRF_LAUNCH("graph_chan_max", s, k_chan_max_final<<<1, 64 * 3, 0, s>>>(pm, G->mx));
  const long nfeat = (long)g.Np * nf;
  MRF_LAUNCH("graph_features", s, k_features<<<ceil_div(nfeat, 256), 256, 0, s>>>(maps, G->mx, g, G->F));
  const int nt = ceil_div(g.Np, kKnnTile);
  MRF_LAUNCH("graph_knn_dist", s, k_knn_dist<<<nt * (nt + 1) / 2, 256, 0, s>>>(G->F, g.Np, nf, nt, G->W));
  const int rc = ceil_div(g.Np, 64);
  const dim3 sg(ceil_div(g.Np, 4));
  if (rc <= 16)
    MRF_LAUNCH("graph_knn_select", s, k_knn_select<16><<<sg, 256, 0, s>>>(G->W, g.Np, K, G->knn, G->knd2, G->kmax));
  else if (rc <= 32)
    MRF_LAUNCH("graph_knn_select", s, k_knn_select<32><<<sg, 256, 0, s>>>(G->W, g.Np, K, G->knn, G->knd2, G->kmax));
  else if (rc <= 64)
    MRF_LAUNCH("graph_knn_select", s, k_knn_select<64><<<sg, 256, 0, s>>>(G->W, g.Np, K, G->knn, G->knd2, G->kmax));
  else
    MRF_LAUNCH("graph_knn_select", s, k_knn_select<128><<<sg, 256, 0, s>>>(G->W, g.Np, K, G->knn, G->knd2, G->kmax));
  if ((long)g.Np * K <= 65536)
    MRF_LAUNCH("graph_sigma", s, k_sigma<<<1, 1024, 0, s>>>(G->knd2, g.Np, K, G->kmax, sigma2, G->scal));
  else
    MRF_LAUNCH("graph_sigma", s, k_sigma_radix<<<1, 1024, 0, s>>>(G->knd2, g.Np, K, G->kmax, sigma2, G->scal));
  const size_t nw = (size_t)g.Np * g.Np;
  MRF_LAUNCH("graph_zero_w", s, k_fill_f<<<1024, 256, 0, s>>>(G->W, nw, 0.f));
  MRF_LAUNCH("graph_scatter_w", s,
             k_scatter_w<<<ceil_div((long)g.Np * K, 256), 256, 0, s>>>(G->knn, G->knd2, g.Np, K, G->kmax, G->scal, G->W));
  MRF_LAUNCH("graph_row_stats", s, k_row_stats<<<g.Np, 256, 0, s>>>(G->W, g.Np, G->cnt, G->deg));
  MRF_LAUNCH("graph_rowptr", s, k_scan_rowptr<<<1, 1024, 0, s>>>(G->cnt, g.Np, G->rowptr, G->deg, G->scal));
  MRF_LAUNCH("graph_csr_fill", s, k_csr_fill<<<g.Np, 256, 0, s>>>(G->W, G->deg, g.Np, G->rowptr, G->col, G->val));
  MRF_CHECK_LAUNCH();
  G->K = K;
  return qc_build(G, s);
}

int lap_frame_chunks(const PatchGeom& g, int L) {
  const int nsub = 256 / (g.s * g.s);
  return ceil_div(L, (long)nsub * kLapFramesPerThread);
}

mrf_status lap_apply_full(const mrf_graph_s* G, const cf* X, cf* Y, int L, hipStream_t s) {
  dim3 grid(G->g.nc * G->g.nc, lap_frame_chunks(G->g, L));
  MRF_LAUNCH("lap_apply", s, k_lap_full<false><<<grid, 256, 0, s>>>(X, Y, nullptr, G->rowptr, G->col, G->val, G->g, L));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// out (device double) = Re<X, S_L X> = Tr(Q(X) L Q(X)^H)
mrf_status lap_quad(mrf_graph_s* G, const cf* X, int L, double* out, hipStream_t s) {
  const PatchGeom& g = G->g;
  const int PP = g.p * g.p;
  if (G->qc) {
    const int ntx = G->ntx, n = G->nslot;
    const int nfc = ceil_div(L, kQcStages * kQcF);
    const int grid = 8 * ntx * ntx * ceil_div(nfc, 8);
    const long nfar = 4L * kQcFarBlocks;
    if ((size_t)(grid + nfar) <= G->npart && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {   // float4 window loads
      const int* pin = G->qc_ptr;
      const int* pout = G->qc_ptr + n + 1;
      const int* nfs = G->qc_fslot + n;
#define MRF_QC(Sv)                                                                                              \
  MRF_LAUNCH("lap_quad", s, k_qc_trace<Sv><<<grid, 64 * kQcWaves, 0, s>>>(X, pin, G->qc_in, G->qc_wd, g, L, ntx, nfc,  \
                                                                         G->part));                             \
  MRF_LAUNCH("lap_quad_far", s,                                                                                 \
             k_qc_far<Sv><<<kQcFarBlocks, 256, 0, s>>>(X, pout, G->qc_out, G->qc_fslot, nfs, g, L, ntx, G->part + grid))
      if (g.s == 4) {
        MRF_QC(4);
      } else {
        MRF_QC(2);
      }
#undef MRF_QC
      MRF_CHECK_LAUNCH();
      return sum_partials2(G->part, grid + nfar, G->part + G->npart, out, s);
    }
  }
  if (PP == 64 || PP == 16) {
    const int fch = PP == 64 ? kQuadFch64 : kQuadFch16;
    const int nchunk = ceil_div(L, fch);
    const size_t nb = (size_t)nchunk * g.Np;
    if (nb > G->npart) return fail(MRF_SHAPE, "laplacian quad: too many frames for the partial-sum buffer");
    const int grid = 8 * ceil_div(g.Np, kQuadWpb) * ceil_div(nchunk, 8);
    const bool vec = g.s % 2 == 0 && g.N % 2 == 0;   // 16-byte aligned pixel pairs
#define MRF_QUAD(PPv, PVv, FCHv) \
  MRF_LAUNCH("lap_quad", s,                                                                                    \
             k_lap_quad_edges<PPv, PVv, FCHv><<<grid, 64 * kQuadWpb, 0, s>>>(X, G->rowptr, G->col, G->val, g, L, nchunk, G->part))
    if (PP == 64 && vec) MRF_QUAD(64, 2, kQuadFch64);
    else if (PP == 64) MRF_QUAD(64, 1, kQuadFch64);
    else if (vec) MRF_QUAD(16, 2, kQuadFch16);
    else MRF_QUAD(16, 1, kQuadFch16);
#undef MRF_QUAD
    MRF_CHECK_LAUNCH();
    return sum_partials2(G->part, (long)nb, G->part + G->npart, out, s);
  }
  dim3 grid(g.nc * g.nc, lap_frame_chunks(g, L));
  const size_t nb = (size_t)grid.x * grid.y;
  if (nb > G->npart) return fail(MRF_SHAPE, "laplacian quad: too many frames for the partial-sum buffer");
  MRF_LAUNCH("lap_quad", s, k_lap_full<true><<<grid, 256, 0, s>>>(X, nullptr, G->part, G->rowptr, G->col, G->val, g, L));
  MRF_LAUNCH("sum_partials", s, k_sum_partials<<<1, 256, 0, s>>>(G->part, (long)nb, out));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status lap_apply_sub(const mrf_graph_s* G, const cf* A, cf* Y, int r, hipStream_t s) {
  if (r > 16) return fail(MRF_SHAPE, "laplacian on subspace coefficients: r must be <= 16");
  if (r % 2 == 0 && (reinterpret_cast<uintptr_t>(A) & 15))
    return fail(MRF_INVALID_ARG, "laplacian on subspace coefficients: A must be 16-byte aligned for even r");
  MRF_LAUNCH("lap_sub", s, k_lap_sub<<<ceil_div(4L * G->g.N * G->g.N, 256), 256, 0, s>>>(A, Y, G->rowptr, G->col, G->val, G->g, r));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

const double* graph_scalars(const mrf_graph_s* G) { return G->scal; }

mrf_status sum_partials(const double* part, long n, double* out, hipStream_t s) {
  MRF_LAUNCH("sum_partials", s, k_sum_partials<<<1, 256, 0, s>>>(part, n, out));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// Sums n partials into out[0] in two fixed-order stages; tmp holds 256 doubles.
mrf_status sum_partials2(const double* part, long n, double* tmp, double* out, hipStream_t s) {
  const long per = (n + 255) / 256;
  MRF_LAUNCH("sum_stage", s, k_sum_stage<<<256, 256, 0, s>>>(part, n, per, tmp));
  MRF_LAUNCH("sum_partials", s, k_sum_partials<<<1, 256, 0, s>>>(tmp, 256, out));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}
const PatchGeom& graph_geom(const mrf_graph_s* G) { return G->g; }
size_t graph_capacity(const mrf_graph_s* G) { return G->cap; }

// Replaces the graph's Laplacian by a given CSR (device arrays, already checked by the caller) and
// its scalars (device doubles: sigma^2, max(L), nnz, 0). Asynchronous device-to-device copies.
mrf_status graph_set_csr(mrf_graph_s* G, const int* rowptr, const int* col, const float* val, int nnz,
                         const double* scal, hipStream_t s) {
  if ((size_t)nnz > G->cap) return fail(MRF_SHAPE, "graph: CSR larger than the graph's capacity");
  MRF_CHECK_HIP(hipMemcpyAsync(G->rowptr, rowptr, (size_t)(G->g.Np + 1) * 4, hipMemcpyDeviceToDevice, s));
  MRF_CHECK_HIP(hipMemcpyAsync(G->col, col, (size_t)nnz * 4, hipMemcpyDeviceToDevice, s));
  MRF_CHECK_HIP(hipMemcpyAsync(G->val, val, (size_t)nnz * 4, hipMemcpyDeviceToDevice, s));
  MRF_CHECK_HIP(hipMemcpyAsync(G->scal, scal, 4 * sizeof(double), hipMemcpyDeviceToDevice, s));
  return qc_build(G, s);
}

}  // namespace mrf

using namespace mrf;

extern "C" mrf_status mrf_graph_create(int n, int p, int s, int k_max, int max_frames, mrf_graph_t* out) {
  clear_error();
  MRF_REQUIRE(out, MRF_INVALID_ARG, "graph_create: null output");
  *out = nullptr;
  PatchGeom g;
  MRF_REQUIRE(make_geom(n, p, s, &g), MRF_SHAPE, "graph_create: need p % s == 0 and (n - p) % s == 0");
  MRF_REQUIRE(s * s <= 256 && p <= 8, MRF_SHAPE, "graph_create: patch side must be <= 8 and s^2 <= 256");
  MRF_REQUIRE(k_max >= 1 && k_max <= 16, MRF_INVALID_ARG, "graph_create: k_max must be in [1, 16]");
  MRF_REQUIRE(max_frames >= 1, MRF_INVALID_ARG, "graph_create: max_frames must be >= 1");
  MRF_REQUIRE(g.Np >= 2 && g.Np <= 8192, MRF_SHAPE, "graph_create: patch count must be in [2, 8192]");
  auto* G = new mrf_graph_s{};
  G->g = g;
  G->kmax = k_max;
  G->nf = 3 * p * p;
  G->cap = (size_t)g.Np * (2 * k_max + 1);
  G->npart = std::max((size_t)g.nc * g.nc * lap_frame_chunks(g, max_frames),
                      (size_t)g.Np * ceil_div(max_frames, 4));
  {  // partials of the cell form of the trace: one per trace block and per out-of-window wave
    const int ntx = ceil_div(g.nc, kQcTB);
    const size_t qc_part = (size_t)8 * ntx * ntx * ceil_div(ceil_div(max_frames, kQcStages * kQcF), 8) +
                           4 * (size_t)kQcFarBlocks;
    G->npart = std::max(G->npart, qc_part);
  }
  bool ok = hipMalloc(&G->F, (size_t)g.Np * G->nf * 4) == hipSuccess &&
            hipMalloc(&G->knn, (size_t)g.Np * k_max * 4) == hipSuccess &&
            hipMalloc(&G->knd2, (size_t)g.Np * k_max * 4) == hipSuccess &&
            hipMalloc(&G->W, (size_t)g.Np * g.Np * 4) == hipSuccess &&
            hipMalloc(&G->rowptr, (size_t)(g.Np + 1) * 4) == hipSuccess &&
            hipMalloc(&G->col, G->cap * 4) == hipSuccess && hipMalloc(&G->val, G->cap * 4) == hipSuccess &&
            hipMalloc(&G->cnt, (size_t)g.Np * 4) == hipSuccess && hipMalloc(&G->deg, (size_t)g.Np * 4) == hipSuccess &&
            hipMalloc(&G->mx, 16) == hipSuccess && hipMalloc(&G->scal, 4 * sizeof(double)) == hipSuccess &&
            hipMalloc(&G->part, (G->npart + 256) * sizeof(double)) == hipSuccess;
  // the cell form of the trace: cells of s x s pixels with p = 2 s, s in {2, 4}, N even
  G->qc = p == 2 * s && (s == 2 || s == 4) && n % 2 == 0;
  if (ok && G->qc) {
    G->ntx = ceil_div(g.nc, kQcTB);
    G->nslot = G->ntx * G->ntx * kQcTB * kQcTB;
    const size_t ns = (size_t)G->nslot;
    ok = hipMalloc(&G->qc_cnt, 2 * ns * sizeof(int)) == hipSuccess &&
         hipMalloc(&G->qc_ptr, 3 * (ns + 1) * sizeof(int)) == hipSuccess &&
         hipMalloc(&G->qc_in, 2 * G->cap * sizeof(int2)) == hipSuccess &&
         hipMalloc(&G->qc_out, 2 * G->cap * sizeof(int2)) == hipSuccess &&
         hipMalloc(&G->qc_wd, ns * sizeof(float)) == hipSuccess &&
         hipMalloc(&G->qc_fslot, (ns + 1) * sizeof(int)) == hipSuccess;
  }
  if (!ok) {
    mrf_graph_destroy(G);
    return fail(MRF_OOM, "graph_create: device allocation failed");
  }
  *out = G;
  return MRF_OK;
}

extern "C" mrf_status mrf_graph_destroy(mrf_graph_t G) {
  clear_error();
  if (!G) return MRF_OK;
  hipFree(G->F); hipFree(G->knn); hipFree(G->knd2); hipFree(G->W); hipFree(G->rowptr); hipFree(G->col);
  hipFree(G->val); hipFree(G->cnt); hipFree(G->deg); hipFree(G->mx); hipFree(G->scal); hipFree(G->part);
  hipFree(G->qc_cnt); hipFree(G->qc_ptr); hipFree(G->qc_in); hipFree(G->qc_out); hipFree(G->qc_wd);
  hipFree(G->qc_fslot);
  delete G;
  return MRF_OK;
}

extern "C" mrf_status mrf_knn_laplacian(mrf_graph_t G, const float* maps, int K, float sigma2, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(G && maps, MRF_INVALID_ARG, "knn_laplacian: null argument");
  MRF_REQUIRE(K >= 1 && K <= G->kmax && K <= G->g.Np - 1, MRF_INVALID_ARG, "knn_laplacian: K must be in [1, min(k_max, Np - 1)]");
  MRF_REQUIRE(sigma2 == sigma2, MRF_INVALID_ARG, "knn_laplacian: sigma2 is NaN");
  return graph_build(G, maps, K, sigma2, s);
}

extern "C" mrf_status mrf_graph_info(mrf_graph_t G, int* np, int* nnz, const int** rowptr, const int** col,
                                     const float** val, double* sigma2, double* lmax, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(G, MRF_INVALID_ARG, "graph_info: null graph");
  double h[4];
  MRF_CHECK_HIP(hipMemcpyAsync(h, G->scal, sizeof h, hipMemcpyDeviceToHost, s));
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  if (np) *np = G->g.Np;
  if (nnz) *nnz = (int)h[2];
  if (rowptr) *rowptr = G->rowptr;
  if (col) *col = G->col;
  if (val) *val = G->val;
  if (sigma2) *sigma2 = h[0];
  if (lmax) *lmax = h[1];
  return MRF_OK;
}

extern "C" mrf_status mrf_laplacian_apply(mrf_graph_t G, const mrf_c64* X, mrf_c64* Y, int L, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(G && X && Y, MRF_INVALID_ARG, "laplacian_apply: null argument");
  MRF_REQUIRE(L >= 1, MRF_INVALID_ARG, "laplacian_apply: L must be >= 1");
  MRF_REQUIRE(X != (const mrf_c64*)Y, MRF_INVALID_ARG, "laplacian_apply: X and Y must not alias");
  return lap_apply_full(G, (const cf*)X, (cf*)Y, L, s);
}

extern "C" mrf_status mrf_laplacian_quad(mrf_graph_t G, const mrf_c64* X, int L, double* out, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(G && X && out, MRF_INVALID_ARG, "laplacian_quad: null argument");
  MRF_REQUIRE(L >= 1, MRF_INVALID_ARG, "laplacian_quad: L must be >= 1");
  return lap_quad(G, (const cf*)X, L, out, s);
}
