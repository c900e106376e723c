// NUFFT pair A / A^H (eq. (1); gradient step eq. (15)) for gfx950.
//
// Forward, per frame (image X_l, N x N -> samples b_l, Ns):
//   k_row_fwd  : each image row is deapodised, zero-padded to G = 2N (centred) and
//                transformed along x (Stockham, in LDS). Writes T[l][y][kx], N x G: only the
//                N non-zero rows of the padded grid are ever formed.
//   k_col_fwd  : one workgroup per (frame, strip of TX grid columns). Loads the strip of T,
//                transforms along y (all G rows, in LDS), then each wave interpolates the
//                samples listed for its tile (TX columns x G/4 rows) with the 6 x 6
//                Kaiser-Bessel taps that fall inside the tile: one partial sum per
//                (sample, tile) entry. The G x G grid never goes to HBM.
//   k_combine  : b[j] = (1/N) * sum of the sample's <= 4 partials, in tile order.
// Adjoint, per frame (the exact transpose of the above):
//   k_col_adj  : one workgroup per (frame, strip). Every grid point of the strip gathers the
//                weighted samples whose 6 x 6 footprint covers it, from its tile's entry list
//                sorted by footprint row: a deterministic spread without atomics. Then the
//                inverse transform along y, keeping only the N rows of the crop.
//   k_row_adj  : inverse transform along x, crop to N columns, deapodise, scale 1/N.
// The plan (host C++) bins each sample into every tile its footprint touches (halo
// duplication), stores the tile-local footprint origin and the 12 separable weights.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "cart.hpp"
#include "common.hpp"
#include "fft.hpp"

namespace mrf {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct alignas(16) Entry {
  int j;        // sample index inside the frame
  int lb;       // tile-local footprint origin: low 16 bits column (signed), high 16 bits row
  float wx[6];  // weights of the 6 column taps
  float wy[6];  // weights of the 6 row taps
  int pad[2];
};
static_assert(sizeof(Entry) == 64, "Entry layout");

}  // namespace mrf

struct mrf_nufft_plan_s {
  int N, G, L, Ns, TX, TY, nstrips, ntiles;  // ntiles per frame = nstrips * 4
  long long E;
  mrf::Entry* ent;
  int* tile_ptr;      // [L * ntiles + 1]
  int4* samp_ent;     // [L * Ns] entry ids of each sample, -1 padded
  float* dinv;        // [N] 1 / phi_hat((x - N/2) / G)
  mrf::cf* tw;        // [G] exp(-2 pi i k / G)
  size_t ws_T, ws_part, ws_bytes;
  // kind 1: Cartesian sampling (mrf_cart_plan_create): G = N, Ns = N * N, mask [L][N][N]; the
  // trajectory tables above are unused
  int kind;
  uint8_t* mask;
};

namespace mrf {

inline bool is_cart(const mrf_nufft_plan_s* p) { return p->kind == 1; }
inline CartOp cart_op(const mrf_nufft_plan_s* p) { return CartOp{p->N, p->L, p->tw, p->mask}; }

// ------------------------------------------------------------------ kernels
// Work distribution of the column kernels: block b handles strip sx of frame chunk c. Blocks are
// dispatched to the 8 XCDs round-robin (XCD = b mod 8); here XCD x takes the chunks c = x (mod 8)
// with all their strips in order. Every XCD then gets the same share of the expensive strips
// that hold the k-space centre (every frame's spiral starts there), and neighbouring strips,
// which share 128-byte lines of T, meet in the same L2.
constexpr int kMaxFramesPerBlock = 1;

// Rows per row-pass group: a radix-8 pass of the group then gives one butterfly per thread
// (for G with factors 3 or 5 the count is rounded down).
__host__ __device__ constexpr int row_rpb(int G) { return kBlock * 8 / G > 0 ? kBlock * 8 / G : 1; }

__device__ inline bool strip_and_chunk(int nstrips, int nchunks, int& sx, int& c) {
  const int b = blockIdx.x;
  const int q = b >> 3;
  sx = q % nstrips;
  c = (q / nstrips) * 8 + (b & 7);
  return c < nchunks;
}

// Row pass, forward: rows of X (deapodised, zero-padded to G) -> T rows. Grid-stride over groups
// of RPB rows; the next group's inputs are loaded into registers while this group transforms.
// A sensitivity map smap (N x N, shared by all frames; null for a single coil) multiplies each
// pixel first: the multi-coil operator of eq. (1) runs this pass once per coil.
template <int G>
__global__ __launch_bounds__(kBlock) void k_row_fwd(const cf* __restrict__ X, cf* __restrict__ T,
                                                    const float* __restrict__ dinv,
                                                    const cf* __restrict__ twg, int nrows,
                                                    const cf* __restrict__ smap) {
  constexpr int N = G / 2;
  constexpr int RPB = row_rpb(G);          // rows per group
  constexpr int PS = 3;                    // one pad element per 8 (LDS banks)
  constexpr int TS = padx<PS>(G) + 1;
  constexpr int PIN = (RPB * N + kBlock - 1) / kBlock;   // non-zero inputs per thread
  __shared__ cf buf[RPB * TS];
  __shared__ cf tw[G];
  const int tid = threadIdx.x;
  for (int i = tid; i < G; i += kBlock) tw[i] = twg[i];
  const int ngroups = (nrows + RPB - 1) / RPB;
  cf pre[PIN];
  auto load = [&](int g) {
#pragma unroll
    for (int i = 0; i < PIN; ++i) {
      const int idx = tid + i * kBlock;
      const long row = (long)g * RPB + idx / N;
      pre[i] = (idx < RPB * N && row < nrows) ? X[row * N + idx % N] : cf{0.f, 0.f};
    }
  };
  int g = blockIdx.x;
  if (g < ngroups) load(g);
  for (; g < ngroups; g += gridDim.x) {
    // place the deapodised inputs at (x - N/2) mod G; the zero padding [N/2, G - N/2) is neither
    // written nor read (the FFT's first pass skips those inputs)
#pragma unroll
    for (int i = 0; i < PIN; ++i) {
      const int idx = tid + i * kBlock;
      if (idx < RPB * N) {
        const int rr = idx / N, x = idx % N;
        const long row = (long)g * RPB + rr;
        const int y = (int)(row % N);
        int n = x - N / 2;
        if (n < 0) n += G;
        const cf v = smap ? cmul(smap[y * N + x], pre[i]) : pre[i];   // coil c sees S_c x
        buf[rr * TS + padx<PS>(n)] = cscale(v, dinv[x] * dinv[y]);
      }
    }
    lds_sync();
    if (g + (int)gridDim.x < ngroups) load(g + gridDim.x);
    lds_fft<G, RPB, 1, TS, false, false, PS, true, false>(buf, tw);
    for (int idx = tid; idx < RPB * G; idx += kBlock) {
      const int rr = idx / G, n = idx % G;
      const long row = (long)g * RPB + rr;
      if (row < nrows) T[row * G + n] = buf[rr * TS + padx<PS>(n)];
    }
    lds_sync();
  }
}

// Row pass, adjoint: T rows -> inverse transform -> crop to N columns, deapodise, scale. With a
// sensitivity map the result is multiplied by its conjugate and, for every coil after the first,
// added to X: the adjoint of the multi-coil operator, one coil per launch.
template <int G>
__global__ __launch_bounds__(kBlock) void k_row_adj(const cf* __restrict__ T, cf* __restrict__ X,
                                                    const float* __restrict__ dinv,
                                                    const cf* __restrict__ twg, int nrows, float scale,
                                                    const cf* __restrict__ smap, int accumulate) {
  constexpr int N = G / 2;
  constexpr int RPB = row_rpb(G);
  constexpr int PS = 3;
  constexpr int TS = padx<PS>(G) + 1;
  constexpr int PIN = (RPB * G + kBlock - 1) / kBlock;
  __shared__ cf buf[RPB * TS];
  __shared__ cf tw[G];
  const int tid = threadIdx.x;
  for (int i = tid; i < G; i += kBlock) tw[i] = twg[i];
  const int ngroups = (nrows + RPB - 1) / RPB;
  cf pre[PIN];
  auto load = [&](int g) {
#pragma unroll
    for (int i = 0; i < PIN; ++i) {
      const int idx = tid + i * kBlock;
      const long row = (long)g * RPB + idx / G;
      pre[i] = (idx < RPB * G && row < nrows) ? T[row * G + idx % G] : cf{0.f, 0.f};
    }
  };
  int g = blockIdx.x;
  if (g < ngroups) load(g);
  for (; g < ngroups; g += gridDim.x) {
#pragma unroll
    for (int i = 0; i < PIN; ++i) {
      const int idx = tid + i * kBlock;
      if (idx < RPB * G) buf[(idx / G) * TS + padx<PS>(idx % G)] = pre[i];
    }
    lds_sync();
    if (g + (int)gridDim.x < ngroups) load(g + gridDim.x);
    lds_fft<G, RPB, 1, TS, false, true, PS, false, true>(buf, tw);   // only the N cropped outputs are stored
    for (int idx = tid; idx < RPB * N; idx += kBlock) {
      const int rr = idx / N, x = idx % N;
      const long row = (long)g * RPB + rr;
      if (row < nrows) {
        int n = x - N / 2;
        if (n < 0) n += G;
        const int y = (int)(row % N);
        cf v = cscale(buf[rr * TS + padx<PS>(n)], dinv[x] * dinv[y] * scale);
        if (smap) v = cconjmul(smap[y * N + x], v);          // coil combine: conj(S_c) A_c^H b_c
        if (accumulate) v = cadd(X[row * N + x], v);         // coils summed in index order
        X[row * N + x] = v;
      }
    }
    lds_sync();
  }
}

// Column pass, forward: per (strip, frame) load the strip of T, transform along y, interpolate.
// Each wave interpolates the entries of its tile (the strip's rows [w G/4, (w+1) G/4)), lane per
// entry, with the taps that fall inside the tile; the sum over a sample's tiles is k_combine.
template <int G, int TX>
__global__ __launch_bounds__(kBlock, 4) void k_col_fwd(const cf* __restrict__ T, const Entry* __restrict__ ent,
                                                    const int* __restrict__ tile_ptr,
                                                    const cf* __restrict__ twg,
                                                    cf* __restrict__ partial, int L, int FC) {
  constexpr int N = G / 2;
  constexpr int P = TX + 1;
  constexpr int TY = G / 4;
  constexpr int NSTRIP = G / TX;
  constexpr int PT = (N * TX + kBlock - 1) / kBlock;
  __shared__ cf S[G * P];   // column TX (the row padding) holds the twiddles tw[k] = S[k P + TX]
  __shared__ int tp[kMaxFramesPerBlock][5];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  int sx, c;
  if (!strip_and_chunk(NSTRIP, (L + FC - 1) / FC, sx, c)) return;
  const int fb = c * FC, fe = min(L, fb + FC);
  const int c0 = sx * TX;
  for (int i = tid; i < G; i += kBlock) S[i * P + TX] = twg[i];
  for (int i = tid; i < (fe - fb) * 5; i += kBlock)
    tp[i / 5][i % 5] = tile_ptr[(size_t)(fb + i / 5) * NSTRIP * 4 + sx * 4 + i % 5];
  lds_sync();
  cf pre[PT];
  Entry en_pre{};
  auto load = [&](int f) {
    const cf* Tf = T + (size_t)f * N * G;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int idx = tid + i * kBlock;
      if (idx < N * TX) pre[i] = Tf[(size_t)(idx / TX) * G + c0 + idx % TX];
    }
    const int e = tp[f - fb][w] + lane;
    if (e < tp[f - fb][w + 1]) en_pre = ent[e];
  };
  load(fb);
  for (int f = fb; f < fe; ++f) {
    // rows [N/2, G - N/2) are the zero padding: the FFT's first pass does not read them
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int idx = tid + i * kBlock;
      if (idx < N * TX) {
        int n = idx / TX - N / 2;
        if (n < 0) n += G;
        S[n * P + idx % TX] = pre[i];
      }
    }
    const Entry first = en_pre;
    lds_sync();
    if (f + 1 < fe) load(f + 1);
    lds_fft<G, TX / 4, P, 1, true, false, 0, true, false, true, P>(S, S + TX);   // per-wave columns, as in k_col_adj
    lds_sync();
    const int e0 = tp[f - fb][w], e1 = tp[f - fb][w + 1];
    const cf* Sw = S + w * TY * P;
    for (int e = e0 + lane; e < e1; e += 64) {
      const Entry en = (e == e0 + lane) ? first : ent[e];
      const int lbx = (short)(en.lb & 0xffff), lby = en.lb >> 16;
      cf acc = {0.f, 0.f};
#pragma unroll
      for (int dy = 0; dy < 6; ++dy) {
        const int row = lby + dy;
        if (row < 0 || row >= TY) continue;
        cf racc = {0.f, 0.f};
#pragma unroll
        for (int dx = 0; dx < 6; ++dx) {
          const int col = lbx + dx;
          if (col < 0 || col >= TX) continue;
          const cf sv = Sw[row * P + col];
          racc.x += en.wx[dx] * sv.x;
          racc.y += en.wx[dx] * sv.y;
        }
        acc.x += en.wy[dy] * racc.x;
        acc.y += en.wy[dy] * racc.y;
      }
      partial[e] = acc;
    }
    lds_sync();
  }
}

// Spread of one tile by one wave, atomics-free and in a fixed order. Lane t owns the grid
// cells (row = R w + t / TX, col = t % TX) of every row window w (R = 64 / TX rows per window)
// and accumulates them in registers. Entries are taken 64 at a time, one per lane; their
// weights are copied to LDS so that a lane can read the tap (dy, dx) it needs. A window only
// visits the entries whose footprint rows reach it: the tile list is sorted by footprint
// row, so that range is found with two ballots over the lanes' footprint rows.
template <int G, int TX>
__device__ inline void spread_tile(const Entry* __restrict__ ent, const cf* __restrict__ rg, int e0, int e1,
                                   const Entry& first, cf first_r, float (*wst)[12], cf* __restrict__ Sw,
                                   int lane) {
  constexpr int TY = G / 4;
  constexpr int R = 64 / TX;
  constexpr int NW = TY / R;
  constexpr int P = TX + 1;
  const int col = lane % TX, rsub = lane / TX;
  cf acc[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) acc[w] = cf{0.f, 0.f};
  for (int base = e0; base < e1; base += 64) {
    const int cnt = min(64, e1 - base);
    int lb = 0x7fff0000;       // rows beyond every window for idle lanes
    cf rv{0.f, 0.f};
    if (lane < cnt) {
      const Entry en = base == e0 ? first : ent[base + lane];
      lb = en.lb;
      rv = base == e0 ? first_r : rg[base + lane];
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        wst[lane][d] = en.wx[d];
        wst[lane][6 + d] = en.wy[d];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int lby = lb >> 16;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int row = w * R + rsub;
      const int a = __popcll(__ballot(lby < w * R - 5));
      const int b = __popcll(__ballot(lby <= w * R + R - 1));
      for (int k = a; k < b; ++k) {
        const int lbk = __builtin_amdgcn_readlane(lb, k);
        const int dy = row - (lbk >> 16), dx = col - (short)(lbk & 0xffff);
        const float rx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rv.x), k));
        const float ry = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rv.y), k));
        if (dy >= 0 && dy < 6 && dx >= 0 && dx < 6) {
          const float wt = wst[k][6 + dy] * wst[k][dx];
          acc[w].x += wt * rx;
          acc[w].y += wt * ry;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
#pragma unroll
  for (int w = 0; w < NW; ++w) Sw[(w * R + rsub) * P + col] = acc[w];
}

// The same spread for TX = 8 as small dense products on MFMA. The kernel is separable, so a window
// of 16 rows of the wave's quarter strip is S_win = A B with A[row][e] = wy_e(row) (zero outside
// entry e's six rows) and B[e][2 c + part] = wx_e(c) (Re, Im)(r_e)[part]: one 16x16x4 MFMA per
// four entries gives the 16 rows x 8 complex columns. Entries are taken in list order, so the
// sums have a fixed order. Lane l of a K-step reads entry 4 s + l / 16 of the batch: origin and
// value by ds_bpermute from the lane that loaded it, weights from LDS.
template <int G>
__device__ inline void spread_tile_mfma(const Entry* __restrict__ ent, const cf* __restrict__ rg, int e0, int e1,
                                        const Entry& first, cf first_r, float (*wst)[12], cf* __restrict__ Sw,
                                        int lane) {
  constexpr int TY = G / 4, NWIN = TY / 16, P = 9;
  static_assert(NWIN >= 1 && TY % 16 == 0, "16-row windows");
  f32x4 acc[NWIN];
#pragma unroll
  for (int wi = 0; wi < NWIN; ++wi) acc[wi] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int m = lane & 15, kk = lane >> 4;
  const int c = m >> 1, part = m & 1;
  for (int base = e0; base < e1; base += 64) {
    const int cnt = min(64, e1 - base);
    int lb = 0x7fff0000;       // rows beyond every window for idle lanes
    cf rv{0.f, 0.f};
    if (lane < cnt) {
      const Entry en = base == e0 ? first : ent[base + lane];
      lb = en.lb;
      rv = base == e0 ? first_r : rg[base + lane];
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        wst[lane][d] = en.wx[d];
        wst[lane][6 + d] = en.wy[d];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int lby = lb >> 16;
#pragma unroll
    for (int wi = 0; wi < NWIN; ++wi) {
      const int r0 = 16 * wi;
      const int a = __popcll(__ballot(lby < r0 - 5));
      const int b = __popcll(__ballot(lby <= r0 + 15));
      for (int k0 = a; k0 < b; k0 += 4) {
        const int k = k0 + kk;
        const bool valid = k < b;
        const int kc = valid ? k : a;   // an entry of the batch, for in-range reads
        const int lbk = __builtin_amdgcn_ds_bpermute(kc << 2, lb);
        const float rx = __int_as_float(__builtin_amdgcn_ds_bpermute(kc << 2, __float_as_int(rv.x)));
        const float ry = __int_as_float(__builtin_amdgcn_ds_bpermute(kc << 2, __float_as_int(rv.y)));
        const int dy = r0 + m - (lbk >> 16), dx = c - (short)(lbk & 0xffff);
        const bool iny = valid && (unsigned)dy < 6u, inx = valid && (unsigned)dx < 6u;
        const float wy = wst[kc][6 + (iny ? dy : 0)];
        const float wx = wst[kc][inx ? dx : 0];
        const float av = iny ? wy : 0.f;
        const float bv = inx ? wx * (part ? ry : rx) : 0.f;
        acc[wi] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[wi], 0, 0, 0);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  float* Sf = reinterpret_cast<float*>(Sw);
#pragma unroll
  for (int wi = 0; wi < NWIN; ++wi)
#pragma unroll
    for (int e = 0; e < 4; ++e) Sf[((16 * wi + 4 * kk + e) * P + c) * 2 + part] = acc[wi][e];
}

// Column pass, adjoint: per (strip, frame) spread the tile entries into the strip (each wave one
// tile), inverse transform along y, write the N crop rows of the strip to T. The next frame's
// first 64 entries per wave and their residual values are prefetched during the transform.
template <int G, int TX>
__global__ __launch_bounds__(kBlock, 3) void k_col_adj(const cf* __restrict__ rg, const Entry* __restrict__ ent,
                                                    const int* __restrict__ tile_ptr,
                                                    const cf* __restrict__ twg, cf* __restrict__ T,
                                                    int L, int FC) {
  constexpr int N = G / 2;
  constexpr int P = TX + 1;
  constexpr int TY = G / 4;
  constexpr int NSTRIP = G / TX;
  __shared__ cf S[G * P];
  __shared__ cf tw[G];
  __shared__ float wst[4][64][12];
  __shared__ int tp[kMaxFramesPerBlock][5];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  int sx, c;
  if (!strip_and_chunk(NSTRIP, (L + FC - 1) / FC, sx, c)) return;
  const int fb = c * FC, fe = min(L, fb + FC);
  const int c0 = sx * TX;
  for (int i = tid; i < G; i += kBlock) tw[i] = twg[i];
  for (int i = tid; i < (fe - fb) * 5; i += kBlock)
    tp[i / 5][i % 5] = tile_ptr[(size_t)(fb + i / 5) * NSTRIP * 4 + sx * 4 + i % 5];
  lds_sync();
  Entry en_pre{};
  cf r_pre{0.f, 0.f};
  auto load = [&](int f) {
    const int e = tp[f - fb][w] + lane;
    if (e < tp[f - fb][w + 1]) {
      en_pre = ent[e];
      r_pre = rg[e];
    }
  };
  load(fb);
  for (int f = fb; f < fe; ++f) {
    const Entry first = en_pre;
    const cf first_r = r_pre;
    if (f + 1 < fe) load(f + 1);
    if constexpr (TX == 8 && (G / 4) % 16 == 0)
      spread_tile_mfma<G>(ent, rg, tp[f - fb][w], tp[f - fb][w + 1], first, first_r, wst[w], S + w * TY * P, lane);
    else
      spread_tile<G, TX>(ent, rg, tp[f - fb][w], tp[f - fb][w + 1], first, first_r, wst[w], S + w * TY * P, lane);
    lds_sync();
    // each wave transforms its TX/4 columns on its own (no workgroup barrier inside), then the
    // block meets before the cropped rows are stored
    lds_fft<G, TX / 4, P, 1, true, true, 0, false, true, true>(S, tw);   // only the N cropped rows are stored
    lds_sync();
    cf* Tf = T + (size_t)f * N * G;
    for (int idx = tid; idx < N * TX; idx += kBlock) {
      const int y = idx / TX, cc = idx % TX;
      int n = y - N / 2;
      if (n < 0) n += G;
      Tf[(size_t)y * G + c0 + cc] = S[n * P + cc];
    }
    lds_sync();
  }
}

__global__ __launch_bounds__(kBlock) void k_combine(const cf* __restrict__ partial,
                                                    const int4* __restrict__ samp_ent,
                                                    cf* __restrict__ b, long total, float scale) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const int4 e = samp_ent[i];
  cf acc = partial[e.x];
  if (e.y >= 0) acc = cadd(acc, partial[e.y]);
  if (e.z >= 0) acc = cadd(acc, partial[e.z]);
  if (e.w >= 0) acc = cadd(acc, partial[e.w]);
  b[i] = cscale(acc, scale);
}

// r = scale * (sum of partials) - b, and per-block partial sums of |r|^2 (double).
__global__ __launch_bounds__(kBlock) void k_combine_resid(const cf* __restrict__ partial,
                                                          const int4* __restrict__ samp_ent,
                                                          const cf* __restrict__ b, cf* __restrict__ r, long total,
                                                          float scale, double* __restrict__ part) {
  __shared__ double red[kBlock];
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  double q = 0.0;
  if (i < total) {
    const int4 e = samp_ent[i];
    cf acc = partial[e.x];
    if (e.y >= 0) acc = cadd(acc, partial[e.y]);
    if (e.z >= 0) acc = cadd(acc, partial[e.z]);
    if (e.w >= 0) acc = cadd(acc, partial[e.w]);
    const cf bv = b[i];
    const cf d = cf{acc.x * scale - bv.x, acc.y * scale - bv.y};
    r[i] = d;
    q = (double)d.x * d.x + (double)d.y * d.y;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Power-iteration helpers: deterministic start vector, <x, y> and ||y||^2 block partials, scaling.
__global__ void k_hash_fill(cf* __restrict__ x, long n, unsigned seed) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    unsigned h = (unsigned)i * 2654435761u ^ seed * 2246822519u;
    h ^= h >> 15; h *= 2246822519u; h ^= h >> 13; h *= 3266489917u; h ^= h >> 16;
    const unsigned g = h * 747796405u + 2891336453u;
    x[i] = cf{(float)(h & 0xffffff) / 16777216.f - 0.5f, (float)(g & 0xffffff) / 16777216.f - 0.5f};
  }
}

__global__ __launch_bounds__(kBlock) void k_dots(const cf* __restrict__ x, const cf* __restrict__ y, long n,
                                                 double* __restrict__ part) {
  __shared__ double r1[kBlock], r2[kBlock];
  double a = 0.0, b = 0.0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const cf u = x[i], v = y[i];
    a += (double)u.x * v.x + (double)u.y * v.y;
    b += (double)v.x * v.x + (double)v.y * v.y;
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      r1[threadIdx.x] += r1[threadIdx.x + o];
      r2[threadIdx.x] += r2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0];
    part[2 * blockIdx.x + 1] = r2[0];
  }
}

__global__ void k_scale_c(cf* __restrict__ x, long n, const double* __restrict__ nrm2) {
  const float s = (float)(1.0 / sqrt(nrm2[0]));
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] = cscale(x[i], s);
}

__global__ void k_sum_pairs(const double* __restrict__ part, int nb, double* __restrict__ out) {
  double a = 0.0, b = 0.0;
  for (int i = 0; i < nb; ++i) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  out[0] = a;
  out[1] = b;
}

// Copies each sample's value to its tile entries (the transpose of k_combine's sum).
__global__ __launch_bounds__(kBlock) void k_gather_r(const cf* __restrict__ r, const int4* __restrict__ samp_ent,
                                                     cf* __restrict__ rg, long total) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const int4 e = samp_ent[i];
  const cf v = r[i];
  rg[e.x] = v;
  if (e.y >= 0) rg[e.y] = v;
  if (e.z >= 0) rg[e.z] = v;
  if (e.w >= 0) rg[e.w] = v;
}

// ------------------------------------------------------------------ host: plan
namespace {

double kb_beta(int W, int osf) {
  const double a = (double)W / osf, b = osf - 0.5;
  return M_PI * std::sqrt(a * a * b * b - 0.8);
}

double bessel_i0(double z) {  // power series sum (z/2)^{2k} / (k!)^2
  const double q = 0.25 * z * z;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * k);
    sum += term;
    if (term <= 1e-18 * sum) break;
  }
  return sum;
}

double kb_kernel(double t, int W, double beta) {
  const double a = 1.0 - (2.0 * t / W) * (2.0 * t / W);
  return a < 0.0 ? 0.0 : bessel_i0(beta * std::sqrt(a));
}

double kb_ft(double s, int W, double beta) {
  const double a = beta * beta - (M_PI * W * s) * (M_PI * W * s);
  if (a > 0) {
    const double r = std::sqrt(a);
    return W * std::sinh(r) / r;
  }
  if (a < 0) {
    const double r = std::sqrt(-a);
    return W * std::sin(r) / r;
  }
  return W;
}

struct FrameBins {
  std::vector<Entry> ent;           // sorted, grouped by tile
  std::vector<int> count;           // per tile
  std::vector<int> samp_of;         // per entry: sample index (== ent.j)
};

void bin_frame(const float* traj, int l, const mrf_nufft_plan_s& p, double beta, FrameBins& out) {
  const int G = p.G, TX = p.TX, TY = p.TY, W = 6;
  std::vector<std::vector<Entry>> tiles(p.ntiles);
  for (int j = 0; j < p.Ns; ++j) {
    const double ux = (double)traj[2 * ((size_t)l * p.Ns + j) + 0] * G / (2.0 * M_PI);
    const double uy = (double)traj[2 * ((size_t)l * p.Ns + j) + 1] * G / (2.0 * M_PI);
    const long bx = (long)std::floor(ux) - W / 2 + 1;
    const long by = (long)std::floor(uy) - W / 2 + 1;
    Entry e{};
    e.j = j;
    for (int d = 0; d < W; ++d) {
      e.wx[d] = (float)kb_kernel(ux - (double)(bx + d), W, beta);
      e.wy[d] = (float)kb_kernel(uy - (double)(by + d), W, beta);
    }
    // tiles are at least 8 cells wide, so a 6-cell footprint meets at most 2 strips / blocks
    int strips[2], nst = 0, blks[2], nbk = 0;
    for (int d = 0; d < W; ++d) {
      const int s = (int)(((bx + d) % G + G) % G) / TX;
      if (!(nst > 0 && strips[0] == s) && !(nst > 1 && strips[1] == s)) strips[nst++] = s;
      const int b = (int)(((by + d) % G + G) % G) / TY;
      if (!(nbk > 0 && blks[0] == b) && !(nbk > 1 && blks[1] == b)) blks[nbk++] = b;
    }
    for (int a = 0; a < nst; ++a) {
      for (int c = 0; c < nbk; ++c) {
        long lx = ((bx - (long)strips[a] * TX) % G + G) % G;
        if (lx >= G - (W - 1)) lx -= G;
        long ly = ((by - (long)blks[c] * TY) % G + G) % G;
        if (ly >= G - (W - 1)) ly -= G;
        Entry q = e;
        q.lb = (int)((uint32_t)(lx & 0xffff) | ((uint32_t)ly << 16));
        tiles[strips[a] * 4 + blks[c]].push_back(q);
      }
    }
  }
  out.ent.clear();
  out.count.assign(p.ntiles, 0);
  for (int t = 0; t < p.ntiles; ++t) {
    auto& v = tiles[t];
    std::stable_sort(v.begin(), v.end(), [](const Entry& a, const Entry& b) {
      const int ra = a.lb >> 16, rb = b.lb >> 16;
      return ra != rb ? ra < rb : a.j < b.j;
    });
    out.count[t] = (int)v.size();
    out.ent.insert(out.ent.end(), v.begin(), v.end());
  }
}

template <typename F>
void parallel_for(int n, F fn) {
  int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min(nt, n);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (int i = t; i < n; i += nt) fn(i);
    });
  for (auto& x : th) x.join();
}

}  // namespace

static bool supported_g(int G) {
  return G == 32 || G == 64 || G == 128 || G == 256 || G == 384 || G == 512 || G == 640 || G == 1024;
}

}  // namespace mrf

using namespace mrf;

extern "C" mrf_status mrf_nufft_plan_create(const mrf_nufft_desc* d, const float* traj, hipStream_t stream,
                                            mrf_nufft_plan_t* out) {
  clear_error();
  MRF_REQUIRE(d && traj && out, MRF_INVALID_ARG, "nufft_plan_create: null argument");
  *out = nullptr;
  MRF_REQUIRE(d->kb_width == 6, MRF_NOT_SUPPORTED, "nufft_plan_create: kb_width must be 6");
  MRF_REQUIRE(d->oversamp == 2, MRF_NOT_SUPPORTED, "nufft_plan_create: oversamp must be 2");
  MRF_REQUIRE(d->nframes >= 1 && d->nsamp >= 1, MRF_INVALID_ARG, "nufft_plan_create: nframes, nsamp must be >= 1");
  const int N = d->n, G = 2 * N;
  MRF_REQUIRE(N >= 16 && N <= 512 && supported_g(G), MRF_SHAPE,
              "nufft_plan_create: n must be 16, 32, 64, 128, 192, 256, 320 or 512");
  int TX = d->tile_cols ? d->tile_cols : (G <= 32 ? 16 : 8);
  MRF_REQUIRE(TX == 8 || TX == 16 || TX == 32, MRF_INVALID_ARG, "nufft_plan_create: tile_cols must be 0, 8, 16 or 32");
  MRF_REQUIRE(TX <= G / 2 && (long)G * TX <= 8192 && (TX < 32 || G <= 128), MRF_SHAPE,
              "nufft_plan_create: tile_cols too large for this grid");
  MRF_REQUIRE((long)d->nframes * d->nsamp < (1L << 30), MRF_SHAPE, "nufft_plan_create: too many samples");

  auto* p = new mrf_nufft_plan_s{};
  p->N = N; p->G = G; p->L = d->nframes; p->Ns = d->nsamp; p->TX = TX; p->TY = G / 4;
  p->nstrips = G / TX; p->ntiles = p->nstrips * 4;

  const size_t nsamp_tot = (size_t)p->L * p->Ns;
  std::vector<float> htraj(2 * nsamp_tot);
  hipError_t e = hipMemcpyAsync(htraj.data(), traj, htraj.size() * sizeof(float), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    delete p;
    return fail(MRF_DEVICE, std::string("nufft_plan_create: trajectory copy: ") + hipGetErrorString(e));
  }
  for (size_t i = 0; i < htraj.size(); ++i) {
    if (!(htraj[i] >= -(float)M_PI && htraj[i] <= (float)M_PI)) {
      delete p;
      return fail(MRF_INVALID_ARG, "nufft_plan_create: trajectory outside [-pi, pi] or not finite");
    }
  }
  const double beta = kb_beta(6, 2);
  std::vector<FrameBins> bins(p->L);
  parallel_for(p->L, [&](int l) { bin_frame(htraj.data(), l, *p, beta, bins[l]); });

  std::vector<int> tile_ptr((size_t)p->L * p->ntiles + 1);
  long long acc = 0;
  for (int l = 0; l < p->L; ++l)
    for (int t = 0; t < p->ntiles; ++t) {
      tile_ptr[(size_t)l * p->ntiles + t] = (int)acc;
      acc += bins[l].count[t];
    }
  tile_ptr.back() = (int)acc;
  if (acc >= (1LL << 31)) {
    delete p;
    return fail(MRF_SHAPE, "nufft_plan_create: too many tile entries");
  }
  p->E = acc;
  std::vector<Entry> ent((size_t)acc);
  std::vector<int4> samp_ent(nsamp_tot, int4{-1, -1, -1, -1});
  parallel_for(p->L, [&](int l) {
    const size_t base = tile_ptr[(size_t)l * p->ntiles];
    std::copy(bins[l].ent.begin(), bins[l].ent.end(), ent.begin() + base);
    for (size_t k = 0; k < bins[l].ent.size(); ++k) {
      int4& s = samp_ent[(size_t)l * p->Ns + bins[l].ent[k].j];
      const int id = (int)(base + k);
      if (s.x < 0) s.x = id; else if (s.y < 0) s.y = id; else if (s.z < 0) s.z = id; else s.w = id;
    }
    bins[l] = FrameBins{};
  });

  std::vector<float> dinv(N);
  for (int x = 0; x < N; ++x) dinv[x] = (float)(1.0 / kb_ft((double)(x - N / 2) / G, 6, beta));
  std::vector<cf> tw(G);
  for (int k = 0; k < G; ++k) tw[k] = cf{(float)std::cos(-2.0 * M_PI * k / G), (float)std::sin(-2.0 * M_PI * k / G)};

  auto cleanup = [&]() {
    hipFree(p->ent); hipFree(p->tile_ptr); hipFree(p->samp_ent); hipFree(p->dinv); hipFree(p->tw);
    delete p;
  };
  if (hipMalloc(&p->ent, std::max<size_t>(1, ent.size()) * sizeof(Entry)) != hipSuccess ||
      hipMalloc(&p->tile_ptr, tile_ptr.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&p->samp_ent, samp_ent.size() * sizeof(int4)) != hipSuccess ||
      hipMalloc(&p->dinv, N * sizeof(float)) != hipSuccess || hipMalloc(&p->tw, G * sizeof(cf)) != hipSuccess) {
    cleanup();
    return fail(MRF_OOM, "nufft_plan_create: device allocation of plan tables failed");
  }
  e = hipMemcpy(p->ent, ent.data(), ent.size() * sizeof(Entry), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->tile_ptr, tile_ptr.data(), tile_ptr.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->samp_ent, samp_ent.data(), samp_ent.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->dinv, dinv.data(), N * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->tw, tw.data(), G * sizeof(cf), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    cleanup();
    return fail(MRF_DEVICE, std::string("nufft_plan_create: table upload: ") + hipGetErrorString(e));
  }
  p->ws_T = ((size_t)p->L * N * G * sizeof(cf) + 255) & ~(size_t)255;
  p->ws_part = ((size_t)p->E * sizeof(cf) + 255) & ~(size_t)255;
  p->ws_bytes = p->ws_T + p->ws_part;
  *out = p;
  return MRF_OK;
}

extern "C" mrf_status mrf_cart_plan_create(int n, int nframes, const uint8_t* mask, hipStream_t stream,
                                           mrf_nufft_plan_t* out) {
  clear_error();
  MRF_REQUIRE(mask && out, MRF_INVALID_ARG, "cart_plan_create: null argument");
  *out = nullptr;
  MRF_REQUIRE(nframes >= 1, MRF_INVALID_ARG, "cart_plan_create: nframes must be >= 1");
  MRF_REQUIRE(cart_supported(n), MRF_SHAPE, "cart_plan_create: n must be 32, 64, 128, 192, 256, 320, 384 or 512");
  MRF_REQUIRE((long)nframes * n * n < (1L << 31), MRF_SHAPE, "cart_plan_create: too many k-space points");
  auto* p = new mrf_nufft_plan_s{};
  p->kind = 1;
  p->N = n; p->G = n; p->L = nframes; p->Ns = n * n;
  std::vector<cf> tw(n);
  for (int k = 0; k < n; ++k) tw[k] = cf{(float)std::cos(-2.0 * M_PI * k / n), (float)std::sin(-2.0 * M_PI * k / n)};
  const size_t nm = (size_t)nframes * n * n;
  hipError_t e = hipMalloc(&p->tw, n * sizeof(cf));
  if (e == hipSuccess) e = hipMalloc(&p->mask, nm);
  if (e != hipSuccess) {
    hipFree(p->tw); hipFree(p->mask);
    delete p;
    return fail(MRF_OOM, "cart_plan_create: device allocation failed");
  }
  e = hipMemcpy(p->tw, tw.data(), n * sizeof(cf), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpyAsync(p->mask, mask, nm, hipMemcpyDefault, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    hipFree(p->tw); hipFree(p->mask);
    delete p;
    return fail(MRF_DEVICE, std::string("cart_plan_create: upload: ") + hipGetErrorString(e));
  }
  p->ws_T = (nm * sizeof(cf) + 255) & ~(size_t)255;
  p->ws_part = 0;
  p->ws_bytes = p->ws_T;
  *out = p;
  return MRF_OK;
}

extern "C" mrf_status mrf_nufft_plan_destroy(mrf_nufft_plan_t p) {
  clear_error();
  if (!p) return MRF_OK;
  hipFree(p->ent); hipFree(p->tile_ptr); hipFree(p->samp_ent); hipFree(p->dinv); hipFree(p->tw);
  hipFree(p->mask);
  delete p;
  return MRF_OK;
}

extern "C" mrf_status mrf_nufft_workspace_size(mrf_nufft_plan_t p, size_t* bytes) {
  clear_error();
  MRF_REQUIRE(p && bytes, MRF_INVALID_ARG, "nufft_workspace_size: null argument");
  *bytes = p->ws_bytes;
  return MRF_OK;
}

namespace mrf {

// One frame per column block: the blocks holding the k-space centre cost several times the
// others, and many small blocks spread them over the whole chip.
static int frames_per_chunk(const mrf_nufft_plan_s*) { return kMaxFramesPerBlock; }

static int col_blocks(const mrf_nufft_plan_s* p, int FC) {
  const int nchunks = (p->L + FC - 1) / FC;
  return 8 * p->nstrips * ((nchunks + 7) / 8);
}

// Grid of a grid-stride row kernel: as many blocks as the device holds at once (CUs times the
// kernel's resident blocks per CU), so that every block is resident from the start and all take
// the same number of row groups; a larger grid leaves a second round of blocks that stretches the
// kernel by their share of the groups. Queried once per kernel.
template <auto kernel>
static int row_blocks(long ngroups) {
  static const int resident = [] {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess)
      return 2048;
    return std::max(1, ncu) * std::max(1, per);
  }();
  return (int)std::min<long>(ngroups, resident);
}

template <int G, int TX>
static void launch_fwd_g(const mrf_nufft_plan_s* p, const cf* img, cf* T, cf* part, const cf* smap,
                         hipStream_t s) {
  const int nrows = p->L * p->N;
  constexpr int RPB = row_rpb(G);
  const int FC = frames_per_chunk(p);
  MRF_LAUNCH("nufft_row_fwd", s,
             k_row_fwd<G><<<row_blocks<k_row_fwd<G>>((nrows + RPB - 1) / RPB), kBlock, 0, s>>>(img, T, p->dinv,
                                                                                          p->tw, nrows, smap));
  MRF_LAUNCH("nufft_col_fwd", s,
             k_col_fwd<G, TX><<<col_blocks(p, FC), kBlock, 0, s>>>(T, p->ent, p->tile_ptr, p->tw, part, p->L, FC));
}

template <int G, int TX>
static void launch_adj_g(const mrf_nufft_plan_s* p, const cf* ksp, cf* img, cf* T, cf* rg, const cf* smap,
                         int accumulate, hipStream_t s) {
  const int nrows = p->L * p->N;
  constexpr int RPB = row_rpb(G);
  const int FC = frames_per_chunk(p);
  const long total = (long)p->L * p->Ns;
  MRF_LAUNCH("nufft_gather_r", s,
             k_gather_r<<<ceil_div(total, kBlock), kBlock, 0, s>>>(ksp, p->samp_ent, rg, total));
  MRF_LAUNCH("nufft_col_adj", s,
             k_col_adj<G, TX><<<col_blocks(p, FC), kBlock, 0, s>>>(rg, p->ent, p->tile_ptr, p->tw, T, p->L, FC));
  MRF_LAUNCH("nufft_row_adj", s,
             k_row_adj<G><<<row_blocks<k_row_adj<G>>((nrows + RPB - 1) / RPB), kBlock, 0, s>>>(T, img, p->dinv,
                                                                                          p->tw, nrows,
                                                                                          1.0f / p->N, smap,
                                                                                          accumulate));
}

#define MRF_DISPATCH_G_TX(FN, ...)                                                   \
  switch (p->G * 100 + p->TX) {                                                      \
    case 32 * 100 + 8: FN<32, 8>(__VA_ARGS__); break;                                \
    case 32 * 100 + 16: FN<32, 16>(__VA_ARGS__); break;                              \
    case 64 * 100 + 8: FN<64, 8>(__VA_ARGS__); break;                                \
    case 64 * 100 + 16: FN<64, 16>(__VA_ARGS__); break;                              \
    case 64 * 100 + 32: FN<64, 32>(__VA_ARGS__); break;                              \
    case 128 * 100 + 8: FN<128, 8>(__VA_ARGS__); break;                              \
    case 128 * 100 + 16: FN<128, 16>(__VA_ARGS__); break;                            \
    case 128 * 100 + 32: FN<128, 32>(__VA_ARGS__); break;                            \
    case 256 * 100 + 8: FN<256, 8>(__VA_ARGS__); break;                              \
    case 256 * 100 + 16: FN<256, 16>(__VA_ARGS__); break;                            \
    case 384 * 100 + 8: FN<384, 8>(__VA_ARGS__); break;                              \
    case 384 * 100 + 16: FN<384, 16>(__VA_ARGS__); break;                            \
    case 512 * 100 + 8: FN<512, 8>(__VA_ARGS__); break;                              \
    case 640 * 100 + 8: FN<640, 8>(__VA_ARGS__); break;                              \
    case 512 * 100 + 16: FN<512, 16>(__VA_ARGS__); break;                            \
    case 1024 * 100 + 8: FN<1024, 8>(__VA_ARGS__); break;                            \
    default: return fail(MRF_SHAPE, "nufft: unsupported grid / tile combination");  \
  }

// The row passes alone, for any grid of the dispatch list (used by the Toeplitz normal operator):
// T [nrows][G] = FFT_x of the rows of X [nrows][G/2] (times dinv, zero-padded, centred), and its
// transpose X [nrows][G/2] (+)= crop of the inverse FFT times dinv times scale.
template <int G>
static void rows_fwd_g(const cf* X, cf* T, const float* dinv, const cf* tw, int nrows, hipStream_t s) {
  constexpr int RPB = row_rpb(G);
  MRF_LAUNCH("toeplitz_row_fwd", s,
             k_row_fwd<G><<<row_blocks<k_row_fwd<G>>((nrows + RPB - 1) / RPB), kBlock, 0, s>>>(X, T, dinv, tw, nrows,
                                                                                          nullptr));
}

template <int G>
static void rows_adj_g(const cf* T, cf* X, const float* dinv, const cf* tw, int nrows, float scale, hipStream_t s) {
  constexpr int RPB = row_rpb(G);
  MRF_LAUNCH("toeplitz_row_adj", s,
             k_row_adj<G><<<row_blocks<k_row_adj<G>>((nrows + RPB - 1) / RPB), kBlock, 0, s>>>(T, X, dinv, tw, nrows,
                                                                                          scale, nullptr, 0));
}

#define MRF_DISPATCH_G(FN, ...)                                                  \
  switch (G) {                                                                   \
    case 32: FN<32>(__VA_ARGS__); break;                                         \
    case 64: FN<64>(__VA_ARGS__); break;                                         \
    case 128: FN<128>(__VA_ARGS__); break;                                       \
    case 256: FN<256>(__VA_ARGS__); break;                                       \
    case 384: FN<384>(__VA_ARGS__); break;                                       \
    case 512: FN<512>(__VA_ARGS__); break;                                       \
    case 640: FN<640>(__VA_ARGS__); break;                                       \
    case 1024: FN<1024>(__VA_ARGS__); break;                                     \
    default: return fail(MRF_SHAPE, "row pass: unsupported grid");              \
  }

mrf_status rows_fwd_padded(int G, const cf* X, cf* T, const float* dinv, const cf* tw, int nrows, hipStream_t s) {
  MRF_DISPATCH_G(rows_fwd_g, X, T, dinv, tw, nrows, s);
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status rows_adj_cropped(int G, const cf* T, cf* X, const float* dinv, const cf* tw, int nrows, float scale,
                            hipStream_t s) {
  MRF_DISPATCH_G(rows_adj_g, T, X, dinv, tw, nrows, scale, s);
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

mrf_status nufft_fwd_partials(const mrf_nufft_plan_s* p, const cf* img, void* ws, hipStream_t s,
                              const cf* smap = nullptr) {
  cf* T = (cf*)ws;
  cf* part = (cf*)((char*)ws + p->ws_T);
  MRF_DISPATCH_G_TX(launch_fwd_g, p, img, T, part, smap, s);
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

const cf* nufft_partials(const mrf_nufft_plan_s* p, void* ws) { return (const cf*)((char*)ws + p->ws_T); }

mrf_status sum_partials(const double* part, long n, double* out, hipStream_t s);

long nufft_resid_blocks(const mrf_nufft_plan_s* p) {
  return is_cart(p) ? cart_part_blocks(p->N, p->L) : ceil_div((long)p->L * p->Ns, kBlock);
}

// r = A img - b and rn2 (device double) = ||r||^2; part needs nufft_resid_blocks doubles per coil.
// With ncoils >= 1 sensitivity maps (smaps [ncoils][N][N]) A is the multi-coil operator of eq. (1):
// b and r hold ncoils k-space series one after another, and ||r||^2 sums over all of them in one
// fixed-order reduction of the coils' block partials.
mrf_status nufft_residual(const mrf_nufft_plan_s* p, const cf* img, const cf* b, cf* r, void* ws, double* part,
                          double* rn2, hipStream_t s, const cf* smaps, int ncoils) {
  const long total = (long)p->L * p->Ns, nb = nufft_resid_blocks(p);
  const long nc = smaps ? ncoils : 1;
  if (is_cart(p)) {
    for (long c = 0; c < nc; ++c) {
      mrf_status st = cart_resid(cart_op(p), img, b + c * total, r + c * total, (cf*)ws, part + c * nb,
                                 smaps ? smaps + c * p->N * p->N : nullptr, s);
      if (st != MRF_OK) return st;
    }
    return sum_partials(part, nc * nb, rn2, s);
  }
  for (long c = 0; c < nc; ++c) {
    mrf_status st = nufft_fwd_partials(p, img, ws, s, smaps ? smaps + c * p->N * p->N : nullptr);
    if (st != MRF_OK) return st;
    MRF_LAUNCH("nufft_combine_resid", s,
               k_combine_resid<<<ceil_div(total, kBlock), kBlock, 0, s>>>(nufft_partials(p, ws), p->samp_ent,
                                                                          b + c * total, r + c * total, total,
                                                                          1.0f / p->N, part + c * nb));
    MRF_CHECK_LAUNCH();
  }
  return sum_partials(part, nc * nb, rn2, s);
}

int nufft_n(const mrf_nufft_plan_s* p) { return p->N; }
int nufft_frames(const mrf_nufft_plan_s* p) { return p->L; }
int nufft_nsamp(const mrf_nufft_plan_s* p) { return p->Ns; }
size_t nufft_ws_bytes(const mrf_nufft_plan_s* p) { return p->ws_bytes; }
const int4* nufft_samp_ent(const mrf_nufft_plan_s* p) { return p->samp_ent; }

mrf_status nufft_adj_impl(const mrf_nufft_plan_s* p, const cf* ksp, cf* img, void* ws, hipStream_t s,
                          const cf* smap = nullptr, int accumulate = 0) {
  if (is_cart(p)) return cart_adj(cart_op(p), ksp, img, (cf*)ws, smap, accumulate, s);
  cf* T = (cf*)ws;
  cf* rg = (cf*)((char*)ws + p->ws_T);
  MRF_DISPATCH_G_TX(launch_adj_g, p, ksp, img, T, rg, smap, accumulate, s);
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// img = sum_c conj(S_c) A^H ksp_c over the coils in index order (the adjoint of eq. (1)'s F_u C);
// smaps null: the single-coil adjoint.
mrf_status nufft_adj_coils(const mrf_nufft_plan_s* p, const cf* ksp, cf* img, void* ws, hipStream_t s,
                           const cf* smaps, int ncoils) {
  if (!smaps) return nufft_adj_impl(p, ksp, img, ws, s);
  const long total = (long)p->L * p->Ns;
  for (long c = 0; c < ncoils; ++c) {
    mrf_status st = nufft_adj_impl(p, ksp + c * total, img, ws, s, smaps + c * p->N * p->N, c > 0);
    if (st != MRF_OK) return st;
  }
  return MRF_OK;
}

}  // namespace mrf

extern "C" mrf_status mrf_nufft_fwd(mrf_nufft_plan_t p, const mrf_c64* img, mrf_c64* ksp, void* ws, size_t ws_bytes,
                                    hipStream_t s) {
  clear_error();
  MRF_REQUIRE(p && img && ksp, MRF_INVALID_ARG, "nufft_fwd: null argument");
  MRF_REQUIRE(ws && ws_bytes >= p->ws_bytes, MRF_WORKSPACE, "nufft_fwd: workspace missing or too small");
  if (is_cart(p)) return cart_fwd(cart_op(p), (const cf*)img, (cf*)ksp, (cf*)ws, nullptr, s);
  mrf_status st = nufft_fwd_partials(p, (const cf*)img, ws, s);
  if (st != MRF_OK) return st;
  const long total = (long)p->L * p->Ns;
  MRF_LAUNCH("nufft_combine", s,
             k_combine<<<ceil_div(total, kBlock), kBlock, 0, s>>>(nufft_partials(p, ws), p->samp_ent, (cf*)ksp,
                                                                  total, 1.0f / p->N));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

extern "C" mrf_status mrf_nufft_adj(mrf_nufft_plan_t p, const mrf_c64* ksp, mrf_c64* img, void* ws, size_t ws_bytes,
                                    hipStream_t s) {
  clear_error();
  MRF_REQUIRE(p && img && ksp, MRF_INVALID_ARG, "nufft_adj: null argument");
  MRF_REQUIRE(ws && ws_bytes >= p->ws_bytes, MRF_WORKSPACE, "nufft_adj: workspace missing or too small");
  return nufft_adj_impl(p, (const cf*)ksp, (cf*)img, ws, s);
}

extern "C" mrf_status mrf_nufft_fwd_mc(mrf_nufft_plan_t p, const mrf_c64* smaps, int ncoils, const mrf_c64* img,
                                       mrf_c64* ksp, void* ws, size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(p && smaps && img && ksp, MRF_INVALID_ARG, "nufft_fwd_mc: null argument");
  MRF_REQUIRE(ncoils >= 1, MRF_INVALID_ARG, "nufft_fwd_mc: ncoils must be >= 1");
  MRF_REQUIRE(ws && ws_bytes >= p->ws_bytes, MRF_WORKSPACE, "nufft_fwd_mc: workspace missing or too small");
  const long total = (long)p->L * p->Ns;
  for (long c = 0; c < ncoils; ++c) {
    if (is_cart(p)) {
      mrf_status st = cart_fwd(cart_op(p), (const cf*)img, (cf*)ksp + c * total, (cf*)ws,
                               (const cf*)smaps + c * p->N * p->N, s);
      if (st != MRF_OK) return st;
      continue;
    }
    mrf_status st = nufft_fwd_partials(p, (const cf*)img, ws, s, (const cf*)smaps + c * p->N * p->N);
    if (st != MRF_OK) return st;
    MRF_LAUNCH("nufft_combine", s,
               k_combine<<<ceil_div(total, kBlock), kBlock, 0, s>>>(nufft_partials(p, ws), p->samp_ent,
                                                                    (cf*)ksp + c * total, total, 1.0f / p->N));
    MRF_CHECK_LAUNCH();
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_nufft_adj_mc(mrf_nufft_plan_t p, const mrf_c64* smaps, int ncoils, const mrf_c64* ksp,
                                       mrf_c64* img, void* ws, size_t ws_bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(p && smaps && img && ksp, MRF_INVALID_ARG, "nufft_adj_mc: null argument");
  MRF_REQUIRE(ncoils >= 1, MRF_INVALID_ARG, "nufft_adj_mc: ncoils must be >= 1");
  MRF_REQUIRE(ws && ws_bytes >= p->ws_bytes, MRF_WORKSPACE, "nufft_adj_mc: workspace missing or too small");
  return nufft_adj_coils(p, (const cf*)ksp, (cf*)img, ws, s, (const cf*)smaps, ncoils);
}

extern "C" mrf_status mrf_nufft_opnorm(mrf_nufft_plan_t p, int iters, unsigned seed, double* lam, hipStream_t s) {
  return mrf_nufft_opnorm_mc(p, nullptr, 0, iters, seed, lam, s);
}

extern "C" mrf_status mrf_nufft_opnorm_mc(mrf_nufft_plan_t p, const mrf_c64* smaps, int ncoils, int iters,
                                          unsigned seed, double* lam, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(p && lam && iters >= 1, MRF_INVALID_ARG, "nufft_opnorm: null argument or iters < 1");
  MRF_REQUIRE(!smaps || ncoils >= 1, MRF_INVALID_ARG, "nufft_opnorm: ncoils must be >= 1 with sensitivity maps");
  const long nimg = (long)p->L * p->N * p->N, nksp = (long)p->L * p->Ns * (smaps ? ncoils : 1);
  cf *x = nullptr, *y = nullptr, *k = nullptr;
  void* ws = nullptr;
  double* d = nullptr;
  const int nb = 1024;
  auto cleanup = [&]() { hipFree(x); hipFree(y); hipFree(k); hipFree(ws); hipFree(d); };
  if (hipMalloc(&x, nimg * 8) != hipSuccess || hipMalloc(&y, nimg * 8) != hipSuccess ||
      hipMalloc(&k, nksp * 8) != hipSuccess || hipMalloc(&ws, p->ws_bytes) != hipSuccess ||
      hipMalloc(&d, (2 * nb + 4) * sizeof(double)) != hipSuccess) {
    cleanup();
    return fail(MRF_OOM, "nufft_opnorm: device allocation failed");
  }
  mrf_status st = MRF_OK;
  double h[2] = {0, 0};
  k_hash_fill<<<1024, 256, 0, s>>>(x, nimg, seed);
  k_dots<<<nb, kBlock, 0, s>>>(x, x, nimg, d);
  k_sum_pairs<<<1, 1, 0, s>>>(d, nb, d + 2 * nb);
  k_scale_c<<<1024, 256, 0, s>>>(x, nimg, d + 2 * nb + 1);
  for (int it = 0; it < iters && st == MRF_OK; ++it) {
    if (smaps) {
      st = mrf_nufft_fwd_mc(p, smaps, ncoils, (const mrf_c64*)x, (mrf_c64*)k, ws, p->ws_bytes, s);
      if (st == MRF_OK) st = mrf_nufft_adj_mc(p, smaps, ncoils, (const mrf_c64*)k, (mrf_c64*)y, ws, p->ws_bytes, s);
    } else {
      st = mrf_nufft_fwd(p, (const mrf_c64*)x, (mrf_c64*)k, ws, p->ws_bytes, s);
      if (st == MRF_OK) st = mrf_nufft_adj(p, (const mrf_c64*)k, (mrf_c64*)y, ws, p->ws_bytes, s);
    }
    if (st != MRF_OK) break;
    k_dots<<<nb, kBlock, 0, s>>>(x, y, nimg, d);               // <x, y> (x unit norm), ||y||^2
    k_sum_pairs<<<1, 1, 0, s>>>(d, nb, d + 2 * nb);
    std::swap(x, y);
    k_scale_c<<<1024, 256, 0, s>>>(x, nimg, d + 2 * nb + 1);   // x = y / ||y||
  }
  if (st == MRF_OK) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, d + 2 * nb, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(MRF_DEVICE, std::string("nufft_opnorm: ") + hipGetErrorString(e));
  }
  cleanup();
  if (st == MRF_OK) *lam = h[0];
  return st;
}

// Autotuner: times the forward + adjoint pair of the trajectory for every strip width the grid
// allows (the spread tile is TX columns by G/4 rows) and returns the fastest. The entry order
// inside a tile is fixed by the design: the atomics-free spread finds each row window's entries
// with two ballots, which needs them sorted by footprint row.
extern "C" mrf_status mrf_nufft_autotune(const mrf_nufft_desc* d, const float* traj, int reps, int* best_tile_cols,
                                         float* pair_ms, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(d && traj && best_tile_cols && reps >= 1, MRF_INVALID_ARG, "nufft_autotune: bad argument");
  const int cand[3] = {8, 16, 32};
  const long nimg = (long)d->nframes * d->n * d->n, nksp = (long)d->nframes * d->nsamp;
  cf *x = nullptr, *k = nullptr;
  void* ws = nullptr;
  size_t ws_have = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    hipFree(x); hipFree(k); hipFree(ws);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  if (hipMalloc(&x, nimg * 8) != hipSuccess || hipMalloc(&k, nksp * 8) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(MRF_OOM, "nufft_autotune: device allocation failed");
  }
  k_hash_fill<<<1024, 256, 0, s>>>(x, nimg, 7u);
  float best = -1.f;
  int best_tx = 0;
  for (int c = 0; c < 3; ++c) {
    if (pair_ms) pair_ms[c] = -1.f;
    const int G = 2 * d->n, TX = cand[c];
    if (!(TX <= G / 2 && (long)G * TX <= 8192 && (TX < 32 || G <= 128))) continue;
    bool dispatched = false;
    switch (G * 100 + TX) {
      case 32 * 100 + 8: case 32 * 100 + 16: case 64 * 100 + 8: case 64 * 100 + 16: case 64 * 100 + 32:
      case 128 * 100 + 8: case 128 * 100 + 16: case 128 * 100 + 32: case 256 * 100 + 8: case 256 * 100 + 16:
      case 384 * 100 + 8: case 384 * 100 + 16: case 512 * 100 + 8: case 512 * 100 + 16: case 640 * 100 + 8:
      case 1024 * 100 + 8:
        dispatched = true;
        break;
      default:
        break;
    }
    if (!dispatched) continue;
    mrf_nufft_desc dc = *d;
    dc.tile_cols = TX;
    mrf_nufft_plan_t p = nullptr;
    mrf_status st = mrf_nufft_plan_create(&dc, traj, s, &p);
    if (st != MRF_OK) {
      cleanup();
      return st;
    }
    if (p->ws_bytes > ws_have) {
      hipFree(ws);
      ws = nullptr;
      if (hipMalloc(&ws, p->ws_bytes) != hipSuccess) {
        mrf_nufft_plan_destroy(p);
        cleanup();
        return fail(MRF_OOM, "nufft_autotune: workspace allocation failed");
      }
      ws_have = p->ws_bytes;
    }
    st = mrf_nufft_fwd(p, (const mrf_c64*)x, (mrf_c64*)k, ws, ws_have, s);
    if (st == MRF_OK) st = mrf_nufft_adj(p, (const mrf_c64*)k, (mrf_c64*)x, ws, ws_have, s);
    hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == MRF_OK; ++r) {
      st = mrf_nufft_fwd(p, (const mrf_c64*)x, (mrf_c64*)k, ws, ws_have, s);
      if (st == MRF_OK) st = mrf_nufft_adj(p, (const mrf_c64*)k, (mrf_c64*)x, ws, ws_have, s);
    }
    hipEventRecord(e1, s);
    float ms = 0.f;
    hipError_t he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    mrf_nufft_plan_destroy(p);
    if (st != MRF_OK) {
      cleanup();
      return st;
    }
    if (he != hipSuccess) {
      cleanup();
      return fail(MRF_DEVICE, std::string("nufft_autotune: ") + hipGetErrorString(he));
    }
    ms /= reps;
    if (pair_ms) pair_ms[c] = ms;
    if (best < 0.f || ms < best) {
      best = ms;
      best_tx = TX;
    }
  }
  cleanup();
  MRF_REQUIRE(best_tx > 0, MRF_SHAPE, "nufft_autotune: no strip width fits this grid");
  *best_tile_cols = best_tx;
  return MRF_OK;
}
