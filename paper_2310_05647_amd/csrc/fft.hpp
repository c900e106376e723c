// Stockham auto-sort FFT on data resident in LDS, for power-of-two lengths 32..1024.
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

// Radix schedule: radix-8 passes, then one radix-4 or radix-2 pass when log2(G) % 3 != 0.
template <int G>
struct FftPlan {
  static constexpr int log2g = (G == 32) ? 5 : (G == 64) ? 6 : (G == 128) ? 7 : (G == 256) ? 8
                             : (G == 512) ? 9 : (G == 1024) ? 10 : -1;
  static_assert(log2g > 0, "unsupported FFT length");
  static constexpr int n8 = log2g / 3;
  static constexpr int tail = 1 << (log2g % 3);   // 1, 2 or 4
  static constexpr int npass = n8 + (tail > 1 ? 1 : 0);
  __host__ __device__ static constexpr int radix(int p) { return p < n8 ? 8 : tail; }
};

template <bool INV>
__device__ inline cf mul_i(cf a) {  // a * (-i) forward, a * (+i) inverse
  return INV ? cf{-a.y, a.x} : cf{a.y, -a.x};
}

template <int R, bool INV>
__device__ inline void dft_regs(cf* v) {
  if constexpr (R == 2) {
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

// One Stockham pass on NT transforms in LDS. CFAST: consecutive threads take consecutive
// transforms (strip layout, ES > 1); otherwise consecutive butterflies (row layout, ES == 1).
template <int G, int R, int NT, int ES, int TS, bool CFAST, bool INV>
__device__ inline void stockham_pass(cf* buf, const cf* tw, int Ns) {
  constexpr int NB = G / R;                 // butterflies per transform
  constexpr int TB = NB * NT;               // butterflies per pass
  constexpr int PER = (TB + kBlock - 1) / kBlock;
  const int tid = threadIdx.x;
  cf v[PER][R];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int id = tid + b * kBlock;
    if (TB % kBlock == 0 || id < TB) {
      const int c = CFAST ? id % NT : id / NB;
      const int j = CFAST ? id / NT : id % NB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[(j + r * NB) * ES + c * TS];
    }
  }
  lds_sync();
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int id = tid + b * kBlock;
    if (TB % kBlock == 0 || id < TB) {
      const int c = CFAST ? id % NT : id / NB;
      const int j = CFAST ? id / NT : id % NB;
      const int k = j % Ns;
      const int step = G / (Ns * R);
      if (Ns > 1) {   // the first pass has only unit twiddles
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cf t = tw[(k * r * step) & (G - 1)];
          if (INV) t.y = -t.y;
          v[b][r] = cmul(v[b][r], t);
        }
      }
      dft_regs<R, INV>(v[b]);
      const int d = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(d + r * Ns) * ES + c * TS] = v[b][r];
    }
  }
  lds_sync();
}

// Full in-LDS FFT of NT transforms of length G. tw[k] = exp(-2 pi i k / G) in LDS.
template <int G, int NT, int ES, int TS, bool CFAST, bool INV>
__device__ inline void lds_fft(cf* buf, const cf* tw) {
  using P = FftPlan<G>;
  int Ns = 1;
#pragma unroll
  for (int p = 0; p < P::npass; ++p) {
    if (P::radix(p) == 8) stockham_pass<G, 8, NT, ES, TS, CFAST, INV>(buf, tw, Ns);
    else if (P::radix(p) == 4) stockham_pass<G, 4, NT, ES, TS, CFAST, INV>(buf, tw, Ns);
    else stockham_pass<G, 2, NT, ES, TS, CFAST, INV>(buf, tw, Ns);
    Ns *= P::radix(p);
  }
}

}  // namespace mrf
