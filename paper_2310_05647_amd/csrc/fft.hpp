// Stockham auto-sort FFT on data resident in LDS, for lengths 2^a 3^b 5^c (32 <= G <= 1024,
// 2^a >= 4): radix-8 passes, one radix-4 or radix-2 pass, then the radix-3 and radix-5 passes.
//
// Pass with radix R over a length-G transform whose finished sub-transforms have span Ns:
//   butterfly j (0 <= j < G/R): v[r] = in[j + r G/R] * w^(k r), k = j mod Ns,
//   w = exp(-+ 2 pi i / (Ns R)); V = DFT_R(v); out[(j / Ns) Ns R + k + r Ns] = V[r].
// All threads of the workgroup cooperate on NT independent transforms stored in one LDS
// array at element address n*ES + c*TS (n: index inside transform c). Every pass loads its
// operands into registers, synchronises, then stores in place (no second buffer).
#pragma once
#include "common.hpp"

namespace mrf {

constexpr int kBlock = 256;

// Workgroup barrier that waits only for this wave's LDS operations, so that global loads
// issued earlier (prefetches) stay in flight across it.
__device__ inline void lds_sync() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0); vmcnt and expcnt left at their maxima
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Ordering of one wave's LDS accesses (a wave's LDS operations execute in order): the wave waits
// for its outstanding LDS reads, and the compiler may not move memory operations across.
__device__ inline void wave_lds_sync() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Radix schedule: radix-8 passes, one radix-4 or radix-2 pass when log2 of the power-of-two
// part is not a multiple of 3, then one pass per factor 3 and per factor 5.
constexpr int count_factor(int g, int f) { return g % f == 0 ? 1 + count_factor(g / f, f) : 0; }
constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
template <int G>
struct FftPlan {
  static constexpr int n3 = count_factor(G, 3);
  static constexpr int n5 = count_factor(G, 5);
  static constexpr int p2 = G / (ipow(3, n3) * ipow(5, n5));
  static constexpr int log2g = ilog2(p2);
  static_assert(p2 >= 4 && (1 << log2g) == p2 && G >= 32 && G <= 1024, "unsupported FFT length");
  static constexpr int n8 = log2g / 3;
  static constexpr int tail = 1 << (log2g % 3);   // 1, 2 or 4
  static constexpr int ntail = tail > 1 ? 1 : 0;
  static constexpr int npass = n8 + ntail + n3 + n5;
  __host__ __device__ static constexpr int radix(int p) {
    return p < n8 ? 8 : p < n8 + ntail ? tail : p < n8 + ntail + n3 ? 3 : 5;
  }
};

template <bool INV>
__device__ inline cf mul_i(cf a) {  // a * (-i) forward, a * (+i) inverse
  return INV ? cf{-a.y, a.x} : cf{a.y, -a.x};
}

template <int R, bool INV>
__device__ inline void dft_regs(cf* v) {
  if constexpr (R == 3) {
    // V_k = sum_n v_n w^{nk}, w = exp(-+ 2 pi i / 3): V_{1,2} = v0 - (v1 + v2)/2 -+ i (sqrt3/2)(v1 - v2)
    constexpr float s3 = 0.86602540378443864676f;
    const cf t1 = cadd(v[1], v[2]);
    const cf t2 = cf{v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y};
    const cf t3 = mul_i<INV>(cscale(csub(v[1], v[2]), s3));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  } else if constexpr (R == 5) {
    // a = v1 + v4, v2 + v3; b = v1 - v4, v2 - v3; V_{1,4} = t1 -+ i u1, V_{2,3} = t2 -+ i u2 with
    // t1 = v0 + c1 a1 + c2 a2, t2 = v0 + c2 a1 + c1 a2, u1 = s1 b1 + s2 b2, u2 = s2 b1 - s1 b2
    constexpr float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    constexpr float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
    const cf a1 = cadd(v[1], v[4]), a2 = cadd(v[2], v[3]);
    const cf b1 = csub(v[1], v[4]), b2 = csub(v[2], v[3]);
    const cf t1 = cf{v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    const cf t2 = cf{v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    const cf u1 = mul_i<INV>(cf{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    const cf u2 = mul_i<INV>(cf{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(t1, u1);
    v[4] = csub(t1, u1);
    v[2] = cadd(t2, u2);
    v[3] = csub(t2, u2);
  } else if constexpr (R == 2) {
    cf a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    cf p0 = cadd(v[0], v[2]), p1 = csub(v[0], v[2]);
    cf p2 = cadd(v[1], v[3]), p3 = mul_i<INV>(csub(v[1], v[3]));
    v[0] = cadd(p0, p2);
    v[2] = csub(p0, p2);
    v[1] = cadd(p1, p3);
    v[3] = csub(p1, p3);
  } else {
    static_assert(R == 8, "radix");
    constexpr float h = 0.70710678118654752440f;
    cf u[4], w[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      u[n] = cadd(v[n], v[n + 4]);
      w[n] = csub(v[n], v[n + 4]);
    }
    // w[n] *= exp(-+ 2 pi i n / 8)
    w[1] = INV ? cf{h * (w[1].x - w[1].y), h * (w[1].x + w[1].y)}
               : cf{h * (w[1].x + w[1].y), h * (w[1].y - w[1].x)};
    w[2] = mul_i<INV>(w[2]);
    w[3] = INV ? cf{-h * (w[3].x + w[3].y), h * (w[3].x - w[3].y)}
               : cf{h * (w[3].y - w[3].x), -h * (w[3].x + w[3].y)};
    dft_regs<4, INV>(u);
    dft_regs<4, INV>(w);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = u[k];
      v[2 * k + 1] = w[k];
    }
  }
}

// Element n of a transform sits at padx<PS>(n) * ES: with PS > 0 one pad element follows every
// 2^PS elements, so that the stride-R stores of the early passes spread over the LDS banks.
template <int PS>
__host__ __device__ constexpr int padx(int n) {
  return PS ? n + (n >> PS) : n;
}

// One Stockham pass on NT transforms in LDS. CFAST: consecutive threads take consecutive
// transforms (strip layout, ES > 1); otherwise consecutive butterflies (row layout, ES == 1).
// ZIN: the inputs n in [G/4, 3G/4) are zero (zero-padded half of a 2x oversampled grid) and are
// not read; only valid for a first pass (Ns = 1) of radix 8, whose butterflies then take r = 0, 1,
// 6, 7. COUT: outputs n in [G/4, 3G/4) are not needed (cropped) and are not stored.
// WAVE: every wave transforms its own NT transforms (wave w: transforms w NT .. w NT + NT - 1)
// and orders its LDS accesses itself, with no workgroup barrier.
template <int G, int R, int NT, int ES, int TS, bool CFAST, bool INV, int PS = 0, bool ZIN = false, bool COUT = false,
          bool WAVE = false, int TWS = 1>
__device__ inline void stockham_pass(cf* buf, const cf* tw, int Ns) {
  static_assert(!ZIN || R == 8, "input pruning needs a radix-8 first pass");
  constexpr int NB = G / R;                 // butterflies per transform
  constexpr int TB = NB * NT;               // butterflies per pass
  constexpr int NTH = WAVE ? 64 : kBlock;   // threads sharing the pass
  constexpr int PER = (TB + NTH - 1) / NTH;
  const int tid = WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  if (WAVE) buf += (threadIdx.x >> 6) * NT * TS;
  cf v[PER][R];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int id = tid + b * NTH;
    if (TB % NTH == 0 || id < TB) {
      const int c = CFAST ? id % NT : id / NB;
      const int j = CFAST ? id / NT : id % NB;
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[b][r] = (ZIN && r >= 2 && r <= 5) ? cf{0.f, 0.f} : buf[padx<PS>(j + r * NB) * ES + c * TS];
    }
  }
  if (WAVE) wave_lds_sync();
  else lds_sync();
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int id = tid + b * NTH;
    if (TB % NTH == 0 || id < TB) {
      const int c = CFAST ? id % NT : id / NB;
      const int j = CFAST ? id / NT : id % NB;
      const int k = j % Ns;
      const int step = G / (Ns * R);
      if (Ns > 1) {   // the first pass has only unit twiddles
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cf t = tw[k * r * step * TWS];   // k r step < G for every pass
          if (INV) t.y = -t.y;
          v[b][r] = cmul(v[b][r], t);
        }
      }
      dft_regs<R, INV>(v[b]);
      const int d = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int o = d + r * Ns;
        if (!COUT || o < G / 4 || o >= 3 * G / 4) buf[padx<PS>(o) * ES + c * TS] = v[b][r];
      }
    }
  }
  if (WAVE) wave_lds_sync();
  else lds_sync();
}

// Full in-LDS FFT of NT transforms of length G. tw[k TWS] = exp(-2 pi i k / G) in LDS.
template <int G, int NT, int ES, int TS, bool CFAST, bool INV, int PS = 0, bool ZIN = false, bool COUT = false,
          bool WAVE = false, int TWS = 1>
__device__ inline void lds_fft(cf* buf, const cf* tw) {
  using P = FftPlan<G>;
  static_assert(!ZIN || P::radix(0) == 8, "input pruning needs a radix-8 first pass");
  int Ns = 1;
#pragma unroll
  for (int p = 0; p < P::npass; ++p) {
    const bool first = p == 0, last = p == P::npass - 1;
    if (P::radix(p) == 8) {
      if (first && last) stockham_pass<G, 8, NT, ES, TS, CFAST, INV, PS, ZIN, COUT, WAVE, TWS>(buf, tw, Ns);
      else if (first) stockham_pass<G, 8, NT, ES, TS, CFAST, INV, PS, ZIN, false, WAVE, TWS>(buf, tw, Ns);
      else if (last) stockham_pass<G, 8, NT, ES, TS, CFAST, INV, PS, false, COUT, WAVE, TWS>(buf, tw, Ns);
      else stockham_pass<G, 8, NT, ES, TS, CFAST, INV, PS, false, false, WAVE, TWS>(buf, tw, Ns);
    } else if (P::radix(p) == 4) {
      if (last) stockham_pass<G, 4, NT, ES, TS, CFAST, INV, PS, false, COUT, WAVE, TWS>(buf, tw, Ns);
      else stockham_pass<G, 4, NT, ES, TS, CFAST, INV, PS, false, false, WAVE, TWS>(buf, tw, Ns);
    } else if (P::radix(p) == 2) {
      if (last) stockham_pass<G, 2, NT, ES, TS, CFAST, INV, PS, false, COUT, WAVE, TWS>(buf, tw, Ns);
      else stockham_pass<G, 2, NT, ES, TS, CFAST, INV, PS, false, false, WAVE, TWS>(buf, tw, Ns);
    } else if (P::radix(p) == 3) {
      if (last) stockham_pass<G, 3, NT, ES, TS, CFAST, INV, PS, false, COUT, WAVE, TWS>(buf, tw, Ns);
      else stockham_pass<G, 3, NT, ES, TS, CFAST, INV, PS, false, false, WAVE, TWS>(buf, tw, Ns);
    } else {
      if (last) stockham_pass<G, 5, NT, ES, TS, CFAST, INV, PS, false, COUT, WAVE, TWS>(buf, tw, Ns);
      else stockham_pass<G, 5, NT, ES, TS, CFAST, INV, PS, false, false, WAVE, TWS>(buf, tw, Ns);
    }
    Ns *= P::radix(p);
  }
}

}  // namespace mrf
