// Full-length dictionary matching Phi_D (eq. (5), Sec. II-B) in FP32, BF16 or FP8 on MFMA, with
// an FP32 re-rank of the best candidates (4 by default, up to 32).
//
// Scores: z_{v,m} = <dn_m, x_v> = sum_l conj(dn_ml) x_vl with the unit-norm atoms dn, so the
// arg-max of |z| is that of |<d_m, x>| / ||d_m||. As a real GEMM with K over real and imaginary
// parts:  Re z = sum (dr xr + di xi),  Im z = sum (dr xi - di xr).
// Every MFMA's K range is split between the two parts: its lane groups q = 0, 1 (of
// q = lane / 16) carry real parts and q = 2, 3 imaginary parts of the same frames. With
// A = atoms (rows m) and B = fingerprints (columns v), Re z is the product of A and B as loaded;
// Im z is the product of A as loaded and B with its two halves swapped, the second of them
// (-xr against di) negated.
//
// Block: 4 waves in a 2 x 2 grid over a 128-atom x 128-fingerprint tile, each wave 64 x 64
// (4 x 4 MFMA tiles, separate real and imaginary accumulators). K advances in chunks whose rows
// are 128 bytes (16 complex FP32 frames interleaved; 32 BF16 frames as [re | im]) or 256 bytes
// (128 FP8 frames as [re | im]), staged in LDS (rows padded by 16 bytes) while the next chunk is
// loaded into registers. A block walks the atom tiles t = g (mod 8) of its group
// g = blockIdx mod 8, so the blocks of one XCD stream the same atom tiles through its L2, and
// keeps per lane a running top-4 (score desc, atom index asc) for each of its 4 fingerprint
// columns (in LDS between atom tiles). The 8 candidate lists of a fingerprint column (32
// candidates) are merged into the block's top-kGroupK, written as the group's partial result;
// k_rerank takes the best `depth` of the 8 groups' candidates and recomputes them exactly in FP32
// from the FP32 atoms.
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "dict.hpp"

namespace mrf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

enum Prec { P_F32 = 0, P_BF16 = 1, P_FP8 = 2, P_BF16X3 = 3 };
constexpr int kGroups = 8;        // atom groups (one per XCD)
constexpr int kTileM = 128;       // atoms per block tile
constexpr int kTileN = 128;       // fingerprints per block tile
constexpr int kE4m3Max = 448;
constexpr int kGroupK = 8;        // candidates per group and fingerprint in the partial results
constexpr int kMaxDepth = 32;     // deepest re-rank

// Per precision: frames per chunk KC, MFMA K-steps per chunk, and the staged row: RB bytes of
// data (RB / 2 of real parts, then RB / 2 of imaginary parts, except FP32's interleaved complex)
// plus 16 bytes of padding.
template <int P>
struct MT;
template <>
struct MT<P_F32> {
  static constexpr int KC = 16;     // frames per chunk
  static constexpr int STEPS = 8;   // MFMA K-steps per chunk (2 frames each)
  static constexpr int RB = 128;
};
template <>
struct MT<P_BF16> {
  static constexpr int KC = 32;
  static constexpr int STEPS = 2;   // 16 frames each
  static constexpr int RB = 128;
};
template <>
struct MT<P_BF16X3> {   // rows as BF16 (hi, lo) pairs: A hi, B hi, A lo, B lo staged
  static constexpr int KC = 32;
  static constexpr int STEPS = 2;
  static constexpr int RB = 128;
};
template <>
struct MT<P_FP8> {
  static constexpr int KC = 128;
  static constexpr int STEPS = 2;   // 64 frames each
  static constexpr int RB = 256;
};
// the dictionary's padded length Lp (a multiple of 128) is a whole number of chunks of every form
static_assert(128 % MT<P_FP8>::KC == 0 && 128 % MT<P_BF16>::KC == 0, "chunks divide 128 frames");

__device__ inline void top4_insert(float (&sc)[4], int (&id)[4], float s, int m) {
  if (!(s > sc[3])) return;   // equal scores keep the earlier (lower) index
  sc[3] = s;
  id[3] = m;
#pragma unroll
  for (int k = 3; k > 0; --k) {
    if (sc[k] > sc[k - 1]) {
      const float ts = sc[k];
      sc[k] = sc[k - 1];
      sc[k - 1] = ts;
      const int ti = id[k];
      id[k] = id[k - 1];
      id[k - 1] = ti;
    }
  }
}

// A: atom rows, B: fingerprint rows, both in the precision's row format (see above); for P_F32
// they are interleaved complex [rows][L]; otherwise [rows][2 Lp] split. sa: FP8 atom scales.
// Partial results: pscore / pidx [Nv][kGroups][4].
// BF16 fits two waves per SIMD (accumulators in the VGPRs, no spills); the other forms need one
template <int P>
__global__ __launch_bounds__(256, P == P_BF16 ? 2 : 1) void k_match_top4(
    const void* __restrict__ A, const float* __restrict__ sa, int M, const void* __restrict__ B, int Nv, int L, int Lp,
    float* __restrict__ pscore, int* __restrict__ pidx, const void* __restrict__ A2 = nullptr,
    const void* __restrict__ B2 = nullptr) {
  typedef MT<P> T;
  constexpr int NGRP = P == P_BF16X3 ? 4 : 2;   // staged row groups: A, B (hi), then A, B (lo)
  constexpr int kRowB = T::RB + 16;             // LDS bytes per staged row
  __shared__ __attribute__((aligned(16))) unsigned char stage[NGRP * kTileM * kRowB];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wa = w >> 1, wf = w & 1;
  const int q = lane >> 4, n16 = lane & 15, h = q >> 1, o = q & 1;
  const int g = blockIdx.x % kGroups;
  const int f0 = (blockIdx.x / kGroups) * kTileN;
  const int ntile = (M + kTileM - 1) / kTileM;
  const int nchunk = P == P_F32 ? (L + T::KC - 1) / T::KC : Lp / T::KC;

  // the running top-4 lists of the thread's 4 fingerprint columns live in LDS between atom tiles
  // (entry (tf, k) of thread t at [4 tf + k][t]), which leaves the registers to the main loop
  __shared__ float lsS[16][256];
  __shared__ int liS[16][256];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    lsS[k][tid] = -1.f;
    liS[k][tid] = -1;
  }

  // register staging of one chunk: NGRP kTileM rows of RB bytes in units of 16 B (P_F32: 8 B)
  constexpr int SEGS = P == P_F32 ? 16 : T::RB / 16;   // units per row
  constexpr int NU = NGRP * kTileM * SEGS / 256;
  static_assert(NGRP * kTileM * SEGS % 256 == 0 && 256 % SEGS == 0, "whole units per thread");
  typedef typename std::conditional<P == P_F32, uint2, uint4>::type U;
  U nxt[NU];
  auto load = [&](int a0, int c) {
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      const int u = tid + 256 * k;
      U v{};
      if constexpr (P == P_F32) {
        const int row = u >> 4, seg = u & 15;
        const int f = c * T::KC + seg;
        const bool isA = row < kTileM;
        const int gr = isA ? a0 + row : f0 + row - kTileM;
        const int lim = isA ? M : Nv;
        const uint2* base = (const uint2*)(isA ? A : B);
        if (gr < lim && f < L) v = base[(size_t)gr * L + f];
        nxt[k] = v;
      } else {
        // u = tid + 256 k: the staged row is RPP k + tid / SEGS (RPP = 256 / SEGS rows per pass),
        // so its group (0 A, 1 B, 2 A lo, 3 B lo) is k / (kTileM / RPP), fixed for each unrolled k
        constexpr int RPP = 256 / SEGS, HS = SEGS / 2;   // HS: units per half (real or imaginary)
        const int seg = tid % SEGS;
        const int grp = k / (kTileM / RPP);
        const int rr = tid / SEGS + RPP * (k % (kTileM / RPP));
        const bool isA = (grp & 1) == 0;
        const int gr = isA ? a0 + rr : f0 + rr;
        const int lim = isA ? M : Nv;
        constexpr int EB = P == P_FP8 ? 1 : 2;   // bytes per element
        const unsigned char* base = (const unsigned char*)(grp == 0 ? A : grp == 1 ? B : grp == 2 ? A2 : B2);
        if (gr < lim) {
          const size_t off = (size_t)gr * 2 * Lp * EB + (size_t)(seg / HS) * Lp * EB + (size_t)c * T::KC * EB +
                             (seg % HS) * 16;
          v = *(const U*)(base + off);
        }
        nxt[k] = v;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      const int u = tid + 256 * k;
      *(U*)(stage + (u / SEGS) * kRowB + (u % SEGS) * sizeof(U)) = nxt[k];
    }
  };

  for (int t = g; t < ntile; t += kGroups) {
    const int a0 = t * kTileM;
    f32x4 re[4][4], im[4][4];
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
      for (int tf = 0; tf < 4; ++tf) {
        re[ta][tf] = f32x4{0.f, 0.f, 0.f, 0.f};
        im[ta][tf] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    load(a0, 0);
    for (int c = 0; c < nchunk; ++c) {
      __syncthreads();   // the previous chunk's reads are done
      store();
      __syncthreads();
      if (c + 1 < nchunk) load(a0, c + 1);   // in flight during this chunk's MFMAs
      const unsigned char* As = stage + (wa * 64 + n16) * kRowB;
      const unsigned char* Bs = stage + (kTileM + wf * 64 + n16) * kRowB;
#pragma unroll
      for (int s = 0; s < T::STEPS; ++s) {
        if constexpr (P == P_F32) {
          const int fb = (2 * s + o) * 8;
          float a[4];
#pragma unroll
          for (int ta = 0; ta < 4; ++ta) a[ta] = *(const float*)(As + ta * 16 * kRowB + fb + 4 * h);
#pragma unroll
          for (int tf = 0; tf < 4; ++tf) {
            const float br = *(const float*)(Bs + tf * 16 * kRowB + fb + 4 * h);
            const float bv = *(const float*)(Bs + tf * 16 * kRowB + fb + 4 * (1 - h));
            const float bi = h ? -bv : bv;   // Im z = dr xi + di (-xr)
#pragma unroll
            for (int ta = 0; ta < 4; ++ta) {
              re[ta][tf] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ta], br, re[ta][tf], 0, 0, 0);
              im[ta][tf] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ta], bi, im[ta][tf], 0, 0, 0);
            }
          }
        } else if constexpr (P == P_BF16) {
          const int ob = s * 32 + o * 16;
          const unsigned sg = h ? 0x80008000u : 0u;
          uint4 a[4];
#pragma unroll
          for (int ta = 0; ta < 4; ++ta) a[ta] = *(const uint4*)(As + ta * 16 * kRowB + h * 64 + ob);
#pragma unroll
          for (int tf = 0; tf < 4; ++tf) {
            const uint4 br = *(const uint4*)(Bs + tf * 16 * kRowB + h * 64 + ob);
            const uint4 bv = *(const uint4*)(Bs + tf * 16 * kRowB + (1 - h) * 64 + ob);
            const uint4 bi = make_uint4(bv.x ^ sg, bv.y ^ sg, bv.z ^ sg, bv.w ^ sg);   // Im z = dr xi + di (-xr)
#pragma unroll
            for (int ta = 0; ta < 4; ++ta) {
              re[ta][tf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[ta]),
                                                                   __builtin_bit_cast(bf16x8, br), re[ta][tf], 0, 0, 0);
              im[ta][tf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[ta]),
                                                                   __builtin_bit_cast(bf16x8, bi), im[ta][tf], 0, 0, 0);
            }
          }
        } else if constexpr (P == P_BF16X3) {
          const int ob = s * 32 + o * 16;
          const unsigned char* As2 = As + 2 * kTileM * kRowB;
          const unsigned char* Bs2 = Bs + 2 * kTileM * kRowB;
          const unsigned sg = h ? 0x80008000u : 0u;
          uint4 a[4], al[4];
#pragma unroll
          for (int ta = 0; ta < 4; ++ta) {
            a[ta] = *(const uint4*)(As + ta * 16 * kRowB + h * 64 + ob);
            al[ta] = *(const uint4*)(As2 + ta * 16 * kRowB + h * 64 + ob);
          }
#pragma unroll
          for (int tf = 0; tf < 4; ++tf) {
            const uint4 br = *(const uint4*)(Bs + tf * 16 * kRowB + h * 64 + ob);
            const uint4 bv = *(const uint4*)(Bs + tf * 16 * kRowB + (1 - h) * 64 + ob);
            const uint4 brl = *(const uint4*)(Bs2 + tf * 16 * kRowB + h * 64 + ob);
            const uint4 bvl = *(const uint4*)(Bs2 + tf * 16 * kRowB + (1 - h) * 64 + ob);
            // Im z = dr xi + di (-xr)
            const uint4 bi = make_uint4(bv.x ^ sg, bv.y ^ sg, bv.z ^ sg, bv.w ^ sg);
            const uint4 bil = make_uint4(bvl.x ^ sg, bvl.y ^ sg, bvl.z ^ sg, bvl.w ^ sg);
#pragma unroll
            for (int ta = 0; ta < 4; ++ta) {
              // hi hi + hi lo + lo hi; the lo lo product is below the accumulation's rounding
              f32x4 r = re[ta][tf], i = im[ta][tf];
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[ta]), __builtin_bit_cast(bf16x8, brl), r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al[ta]), __builtin_bit_cast(bf16x8, br), r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[ta]), __builtin_bit_cast(bf16x8, br), r, 0, 0, 0);
              i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[ta]), __builtin_bit_cast(bf16x8, bil), i, 0, 0, 0);
              i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al[ta]), __builtin_bit_cast(bf16x8, bi), i, 0, 0, 0);
              i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[ta]), __builtin_bit_cast(bf16x8, bi), i, 0, 0, 0);
              re[ta][tf] = r;
              im[ta][tf] = i;
            }
          }
        } else {
          const int ob = s * 64 + o * 32;
          const int sg = h ? (int)0x80808080u : 0;
          i32x8 a[4];
#pragma unroll
          for (int ta = 0; ta < 4; ++ta) {
            const uint4 lo = *(const uint4*)(As + ta * 16 * kRowB + h * 128 + ob);
            const uint4 hi = *(const uint4*)(As + ta * 16 * kRowB + h * 128 + ob + 16);
            a[ta] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
          }
#pragma unroll
          for (int tf = 0; tf < 4; ++tf) {
            const uint4 rlo = *(const uint4*)(Bs + tf * 16 * kRowB + h * 128 + ob);
            const uint4 rhi = *(const uint4*)(Bs + tf * 16 * kRowB + h * 128 + ob + 16);
            const uint4 ilo = *(const uint4*)(Bs + tf * 16 * kRowB + (1 - h) * 128 + ob);
            const uint4 ihi = *(const uint4*)(Bs + tf * 16 * kRowB + (1 - h) * 128 + ob + 16);
            const i32x8 br = {(int)rlo.x, (int)rlo.y, (int)rlo.z, (int)rlo.w, (int)rhi.x, (int)rhi.y, (int)rhi.z, (int)rhi.w};
            // Im z = dr xi + di (-xr)
            const i32x8 bi = i32x8{(int)ilo.x, (int)ilo.y, (int)ilo.z, (int)ilo.w, (int)ihi.x, (int)ihi.y, (int)ihi.z,
                                   (int)ihi.w} ^ sg;
#pragma unroll
            for (int ta = 0; ta < 4; ++ta) {
              re[ta][tf] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[ta], br, re[ta][tf], 0, 0, 0, 0x7f7f7f7f, 0,
                                                                            0x7f7f7f7f);
              im[ta][tf] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[ta], bi, im[ta][tf], 0, 0, 0, 0x7f7f7f7f,
                                                                            0, 0x7f7f7f7f);
            }
          }
        }
      }
    }
    // epilogue: |z|^2 (times the atom's squared scale in FP8) into the running top-4 lists
    float ls[4][4];
    int li[4][4];
#pragma unroll
    for (int tf = 0; tf < 4; ++tf)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ls[tf][k] = lsS[4 * tf + k][tid];
        li[tf][k] = liS[4 * tf + k][tid];
      }
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = a0 + wa * 64 + ta * 16 + 4 * q + i;
        if (m < M) {
          const float s2 = P == P_FP8 ? sa[m] * sa[m] : 1.f;
#pragma unroll
          for (int tf = 0; tf < 4; ++tf) {
            const float sc = (re[ta][tf][i] * re[ta][tf][i] + im[ta][tf][i] * im[ta][tf][i]) * s2;
            top4_insert(ls[tf], li[tf], sc, m);
          }
        }
      }
#pragma unroll
    for (int tf = 0; tf < 4; ++tf)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        lsS[4 * tf + k][tid] = ls[tf][k];
        liS[4 * tf + k][tid] = li[tf][k];
      }
  }
  // merge the 8 lists (2 atom waves x 4 lane groups) of each fingerprint column
  __syncthreads();
  float* cs = (float*)stage;                    // [128][8][4]
  int* ci = (int*)(stage + kTileN * 32 * 4);    // [128][8][4]
#pragma unroll
  for (int tf = 0; tf < 4; ++tf) {
    const int col = wf * 64 + tf * 16 + n16, src = wa * 4 + q;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cs[(col * 8 + src) * 4 + k] = lsS[4 * tf + k][tid];
      ci[(col * 8 + src) * 4 + k] = liS[4 * tf + k][tid];
    }
  }
  __syncthreads();
  if (tid < kTileN && f0 + tid < Nv) {
    constexpr int K = kGroupK;
    float sc[K];
    int id[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      sc[k] = -1.f;
      id[k] = -1;
    }
    for (int j = 0; j < 32; ++j) {
      const float s = cs[tid * 32 + j];
      const int m = ci[tid * 32 + j];
      if (m < 0) continue;
      // insertion with ties broken by the lower index (the lists arrive in no index order)
      if (s > sc[K - 1] || (s == sc[K - 1] && (id[K - 1] < 0 || m < id[K - 1]))) {
        sc[K - 1] = s;
        id[K - 1] = m;
        for (int k = K - 1; k > 0; --k) {
          const bool up = sc[k] > sc[k - 1] || (sc[k] == sc[k - 1] && (id[k - 1] < 0 || id[k] < id[k - 1]));
          if (!up) break;
          const float ts = sc[k];
          sc[k] = sc[k - 1];
          sc[k - 1] = ts;
          const int ti = id[k];
          id[k] = id[k - 1];
          id[k - 1] = ti;
        }
      }
    }
    const size_t oK = ((size_t)(f0 + tid) * kGroups + g) * K;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      pscore[oK + k] = sc[k];
      pidx[oK + k] = id[k];
    }
  }
}

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline float wsumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline unsigned long long wmax64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long u = __shfl_xor(v, o);
    v = u > v ? u : v;
  }
  return v;
}

// One wave per fingerprint: the `depth` best of the 8 groups' kGroupK candidates (score desc,
// index asc; one candidate per lane), then z = <dn_m, x> in FP32 for each, two candidates at a
// time, and the exact arg-max of |z| (ties to the lower index).
__global__ __launch_bounds__(256) void k_rerank(const float* __restrict__ pscore, const int* __restrict__ pidx,
                                                const cf* __restrict__ X, int Nv, int L, const cf* __restrict__ dn,
                                                const float* __restrict__ norms, const float* __restrict__ lut,
                                                int nparam, int depth, int* __restrict__ idx, float* __restrict__ rho,
                                                float* __restrict__ score, float* __restrict__ params,
                                                int* __restrict__ cand) {
  static_assert(kGroups * kGroupK == 64, "one candidate per lane");
  const int v = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (v >= Nv) return;
  unsigned long long key = 0ull;
  {
    const float s = pscore[(size_t)v * 64 + lane];
    const int m = pidx[(size_t)v * 64 + lane];
    if (m >= 0 && s >= 0.f)
      key = ((unsigned long long)__float_as_uint(s) << 32) | (unsigned long long)(0xffffffffu - (unsigned)m);
  }
  // the depth best, in order: lane k keeps the k-th
  int mine = -1;
  for (int k = 0; k < depth; ++k) {
    const unsigned long long best = wmax64(key);
    const int m = best ? (int)(0xffffffffu - (unsigned)(best & 0xffffffffull)) : -1;
    if (lane == k) mine = m;
    if (best && key == best) key = 0ull;
  }
  const cf* x = X + (size_t)v * L;
  int bm = -1;
  float bz = -1.f, bre = 0.f;
  auto take = [&](int m, float zr, float zi) {
    const float az = sqrtf(zr * zr + zi * zi);
    if (az > bz || (az == bz && m < bm)) {
      bz = az;
      bm = m;
      bre = zr;
    }
  };
  for (int k = 0; k < depth; k += 2) {
    const int ma = __shfl(mine, k), mb = k + 1 < depth ? __shfl(mine, k + 1) : -1;
    if (ma < 0) break;   // uniform over the wave; the list is in descending order
    const cf* da = dn + (size_t)ma * L;
    const cf* db = dn + (size_t)(mb >= 0 ? mb : ma) * L;
    float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
    for (int f = lane; f < L; f += 64) {
      const cf a = da[f], b = db[f], xx = x[f];
      ar += a.x * xx.x + a.y * xx.y;
      ai += a.x * xx.y - a.y * xx.x;
      br += b.x * xx.x + b.y * xx.y;
      bi += b.x * xx.y - b.y * xx.x;
    }
    ar = wsumf(ar);
    ai = wsumf(ai);
    br = wsumf(br);
    bi = wsumf(bi);
    take(ma, ar, ai);
    if (mb >= 0) take(mb, br, bi);
  }
  if (lane == 0) {
    idx[v] = bm;
    if (score) score[v] = bm >= 0 ? bz : 0.f;
    if (rho) rho[v] = bm >= 0 ? fmaxf(bre / norms[bm], 0.f) : 0.f;
  }
  if (cand && lane < depth) cand[(size_t)v * depth + lane] = mine;
  if (params && lane < nparam) params[(size_t)v * nparam + lane] = bm >= 0 ? lut[(size_t)bm * nparam + lane] : 0.f;
}

// ------------------------------------------------------------------ row conversions
__device__ inline uint16_t to_bf16(float f) {   // round to nearest even
  const unsigned u = __float_as_uint(f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// One block per row: BF16 copy, and FP8 copy with scale max|component| / 448, of a complex row.
__device__ inline float from_bf16(uint16_t b) { return __uint_as_float((unsigned)b << 16); }

__global__ __launch_bounds__(256) void k_quant_rows(const cf* __restrict__ src, int rows, int L, int Lp,
                                                    uint16_t* __restrict__ d16, uint16_t* __restrict__ d16lo,
                                                    uint8_t* __restrict__ d8, float* __restrict__ s8) {
  __shared__ float red[256];
  const int row = blockIdx.x, t = threadIdx.x;
  const cf* x = src + (size_t)row * L;
  float mx = 0.f;
  for (int f = t; f < L; f += 256) mx = fmaxf(mx, fmaxf(fabsf(x[f].x), fabsf(x[f].y)));
  red[t] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] = fmaxf(red[t], red[t + o]);
    __syncthreads();
  }
  const float sc = red[0] > 0.f ? red[0] / kE4m3Max : 1.f;
  const float isc = 1.f / sc;
  if (t == 0 && s8) s8[row] = sc;
  for (int j = t; j < Lp / 2; j += 256) {
    const int f = 2 * j;
    const cf a = f < L ? x[f] : cf{0.f, 0.f};
    const cf b = f + 1 < L ? x[f + 1] : cf{0.f, 0.f};
    if (d16) {
      uint16_t* r16 = d16 + (size_t)row * 2 * Lp;
      const uint16_t h0 = to_bf16(a.x), h1 = to_bf16(b.x), h2 = to_bf16(a.y), h3 = to_bf16(b.y);
      r16[f] = h0;
      r16[f + 1] = h1;
      r16[Lp + f] = h2;
      r16[Lp + f + 1] = h3;
      if (d16lo) {   // the remainders, exact in FP32, rounded to BF16
        uint16_t* l16 = d16lo + (size_t)row * 2 * Lp;
        l16[f] = to_bf16(a.x - from_bf16(h0));
        l16[f + 1] = to_bf16(b.x - from_bf16(h1));
        l16[Lp + f] = to_bf16(a.y - from_bf16(h2));
        l16[Lp + f + 1] = to_bf16(b.y - from_bf16(h3));
      }
    }
    if (d8) {
      uint8_t* r8 = d8 + (size_t)row * 2 * Lp;
      const int pr = __builtin_amdgcn_cvt_pk_fp8_f32(a.x * isc, b.x * isc, 0, false);
      const int pi = __builtin_amdgcn_cvt_pk_fp8_f32(a.y * isc, b.y * isc, 0, false);
      *(uint16_t*)(r8 + f) = (uint16_t)(pr & 0xffff);
      *(uint16_t*)(r8 + Lp + f) = (uint16_t)(pi & 0xffff);
    }
  }
}

mrf_status quantise_rows(const cf* src, int rows, int L, int Lp, uint16_t* d16, uint16_t* d16lo, uint8_t* d8,
                         float* s8, hipStream_t s) {
  if (rows <= 0) return MRF_OK;
  MRF_LAUNCH("match_quantise", s, k_quant_rows<<<rows, 256, 0, s>>>(src, rows, L, Lp, d16, d16lo, d8, s8));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// [L][Nv] -> [Nv][L] through 32 x 32 LDS tiles.
__global__ __launch_bounds__(256) void k_transpose(const cf* __restrict__ X, int L, int Nv, cf* __restrict__ Y) {
  __shared__ cf tile[32][33];
  const int v0 = blockIdx.x * 32, l0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int l = l0 + k, v = v0 + tx;
    if (l < L && v < Nv) tile[k][tx] = X[(size_t)l * Nv + v];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int v = v0 + k, l = l0 + tx;
    if (l < L && v < Nv) Y[(size_t)v * L + l] = tile[tx][k];
  }
}

struct MatchWs {
  void* rows;      // fingerprint rows in the mode's format
  float* pscore;   // [Nv][kGroups][kGroupK]
  int* pidx;
  size_t bytes;
};
static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
MatchWs match_ws(const mrf_dict_s* D, int Nv, int mode, void* base) {
  MatchWs w{};
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = p ? p + off : nullptr;
    off += al(b);
    return (void*)q;
  };
  const size_t rb = mode == MRF_MATCH_BF16_RERANK4 ? (size_t)Nv * 2 * D->Lp * 2
                    : mode == MRF_MATCH_BF16X3_RERANK ? (size_t)Nv * 2 * D->Lp * 2 * 2
                    : mode == MRF_MATCH_FP8_RERANK4 ? (size_t)Nv * 2 * D->Lp
                                                    : 0;
  w.rows = take(rb);
  w.pscore = (float*)take((size_t)Nv * kGroups * kGroupK * 4);
  w.pidx = (int*)take((size_t)Nv * kGroups * kGroupK * 4);
  w.bytes = off;
  return w;
}

}  // namespace mrf

using namespace mrf;

extern "C" mrf_status mrf_frames_to_voxels(const mrf_c64* X, int L, int Nv, mrf_c64* Y, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(X && Y && X != Y, MRF_INVALID_ARG, "frames_to_voxels: null or aliased argument");
  MRF_REQUIRE(L >= 1 && Nv >= 1, MRF_INVALID_ARG, "frames_to_voxels: bad sizes");
  dim3 grid(ceil_div(Nv, 32), ceil_div(L, 32));
  MRF_LAUNCH("frames_to_voxels", s, k_transpose<<<grid, 256, 0, s>>>((const cf*)X, L, Nv, (cf*)Y));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_match_workspace_size(mrf_dict_t D, int Nv, mrf_match_mode mode, size_t* bytes) {
  clear_error();
  MRF_REQUIRE(D && bytes && Nv >= 1, MRF_INVALID_ARG, "dict_match_workspace_size: bad argument");
  MRF_REQUIRE(mode == MRF_MATCH_FP32 || mode == MRF_MATCH_BF16_RERANK4 || mode == MRF_MATCH_FP8_RERANK4 ||
                  mode == MRF_MATCH_BF16X3_RERANK,
              MRF_NOT_SUPPORTED, "dict_match_workspace_size: mode not supported by this call");
  *bytes = match_ws(D, Nv, mode, nullptr).bytes;
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_match(mrf_dict_t D, const mrf_c64* fp, int Nv, mrf_match_mode mode, int32_t* idx,
                                     float* rho, float* score, float* params, int32_t* cand, void* ws, size_t ws_bytes,
                                     hipStream_t s) {
  return mrf_dict_match_depth(D, fp, Nv, mode, 4, idx, rho, score, params, cand, ws, ws_bytes, s);
}

extern "C" mrf_status mrf_dict_match_depth(mrf_dict_t D, const mrf_c64* fp, int Nv, mrf_match_mode mode, int depth,
                                           int32_t* idx, float* rho, float* score, float* params, int32_t* cand,
                                           void* ws, size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(D && fp && idx, MRF_INVALID_ARG, "dict_match: null argument");
  MRF_REQUIRE(Nv >= 1, MRF_INVALID_ARG, "dict_match: Nv must be >= 1");
  MRF_REQUIRE(depth >= 1 && depth <= kMaxDepth, MRF_INVALID_ARG, "dict_match: the re-rank depth must be in [1, 32]");
  MRF_REQUIRE(mode == MRF_MATCH_FP32 || mode == MRF_MATCH_BF16_RERANK4 || mode == MRF_MATCH_FP8_RERANK4 ||
                  mode == MRF_MATCH_BF16X3_RERANK,
              MRF_NOT_SUPPORTED, "dict_match: mode not supported by this call");
  const MatchWs w = match_ws(D, Nv, mode, ws);
  MRF_REQUIRE(ws && ws_bytes >= w.bytes, MRF_WORKSPACE, "dict_match: workspace too small");
  const int grid = kGroups * ceil_div(Nv, kTileN);
  const cf* X = (const cf*)fp;
  if (mode == MRF_MATCH_FP32) {
    MRF_LAUNCH("match_full_fp32", s,
               k_match_top4<P_F32><<<grid, 256, 0, s>>>(D->dn, nullptr, D->M, X, Nv, D->L, D->Lp, w.pscore, w.pidx));
  } else if (mode == MRF_MATCH_BF16X3_RERANK) {
    uint16_t* hi = (uint16_t*)w.rows;
    uint16_t* lo = hi + (size_t)Nv * 2 * D->Lp;
    MRF_LAUNCH("match_quantise", s, k_quant_rows<<<Nv, 256, 0, s>>>(X, Nv, D->L, D->Lp, hi, lo, nullptr, nullptr));
    MRF_LAUNCH("match_full_bf16x3", s,
               k_match_top4<P_BF16X3><<<grid, 256, 0, s>>>(D->d16, nullptr, D->M, hi, Nv, D->L, D->Lp, w.pscore, w.pidx,
                                                           D->d16lo, lo));
  } else if (mode == MRF_MATCH_BF16_RERANK4) {
    MRF_LAUNCH("match_quantise", s,
               k_quant_rows<<<Nv, 256, 0, s>>>(X, Nv, D->L, D->Lp, (uint16_t*)w.rows, nullptr, nullptr, nullptr));
    MRF_LAUNCH("match_full_bf16", s,
               k_match_top4<P_BF16><<<grid, 256, 0, s>>>(D->d16, nullptr, D->M, w.rows, Nv, D->L, D->Lp, w.pscore, w.pidx));
  } else {
    MRF_LAUNCH("match_quantise", s,
               k_quant_rows<<<Nv, 256, 0, s>>>(X, Nv, D->L, D->Lp, nullptr, nullptr, (uint8_t*)w.rows, nullptr));
    MRF_LAUNCH("match_full_fp8", s,
               k_match_top4<P_FP8><<<grid, 256, 0, s>>>(D->d8, D->s8, D->M, w.rows, Nv, D->L, D->Lp, w.pscore, w.pidx));
  }
  MRF_LAUNCH("match_rerank", s,
             k_rerank<<<ceil_div(Nv, 4), 256, 0, s>>>(w.pscore, w.pidx, X, Nv, D->L, D->dn, D->norms, D->lut, D->nparam,
                                                     depth, idx, rho, score, params, cand));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}
