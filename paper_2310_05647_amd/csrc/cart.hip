// Cartesian acquisition (eq. (1) with pseudo-radial Cartesian sampling, Sec. IV): for frame l,
// A_l X_l = M_l (F X_l), F the unitary centred 2D DFT (the non-Cartesian operator's definition
// with every frequency on the integer grid: k-space point (ky + N/2, kx + N/2) holds frequency
// (kx, ky)), M_l the frame's 0/1 mask; measurements and residuals are dense [L][N][N] arrays.
// Each direction is two passes of length-N FFTs in LDS. The half-length circular shifts of the
// centred transform fold into the load and store indices: position p <-> FFT index
// (p + N/2) mod N, the same map both ways for even N.
//   forward  k_cart_rows<N, false>  X rows (times S_c) -> FFT along x -> T
//            k_cart_cols<N, false>  strips of T -> FFT along y -> 1/N, mask -> ksp, or
//                                   r = A X - b with block partials of ||r||^2
//   adjoint  k_cart_cols<N, true>   strips of ksp times mask -> inverse FFT along y -> T
//            k_cart_rows<N, true>   T rows -> inverse FFT along x -> 1/N, times conj(S_c),
//                                   added over the coils in index order -> X
// Both passes read and write each element once: HBM-bound, 4 L N^2 complex accesses per pass
// pair plus the mask bytes.
#include <hip/hip_runtime.h>

#include "cart.hpp"
#include "common.hpp"
#include "fft.hpp"

namespace mrf {

constexpr int kCartTX = 16;   // columns of one column-pass block (4 per wave)

template <int N>
__host__ __device__ constexpr int cart_shift(int p) {
  return p + N / 2 < N ? p + N / 2 : p - N / 2;
}

template <int N>
__host__ __device__ constexpr int cart_rpb() {
  return kBlock * 8 / N > 0 ? kBlock * 8 / N : 1;
}

// Row pass over RPB rows per block. Forward: out = FFT_x(in * S); inverse: out (+)= conj(S) *
// scale * IFFT_x(in).
template <int N, bool INV>
__global__ __launch_bounds__(kBlock) void k_cart_rows(const cf* __restrict__ in, cf* __restrict__ out,
                                                      const cf* __restrict__ twg, long nrows,
                                                      const cf* __restrict__ smap, int accumulate, float scale) {
  constexpr int RPB = cart_rpb<N>();
  constexpr int PS = 3;                     // one pad element per 8 (LDS banks)
  constexpr int TS = padx<PS>(N) + 1;
  __shared__ cf buf[RPB * TS];
  __shared__ cf tw[N];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += kBlock) tw[i] = twg[i];
  const long row0 = (long)blockIdx.x * RPB;
  for (int idx = tid; idx < RPB * N; idx += kBlock) {
    const int rr = idx / N, p = idx % N;
    const long row = row0 + rr;
    cf v = {0.f, 0.f};
    if (row < nrows) {
      v = in[row * N + p];
      if (!INV && smap) v = cmul(smap[(row % N) * N + p], v);
    }
    buf[rr * TS + padx<PS>(cart_shift<N>(p))] = v;
  }
  lds_sync();
  lds_fft<N, RPB, 1, TS, false, INV, PS>(buf, tw);
  for (int idx = tid; idx < RPB * N; idx += kBlock) {
    const int rr = idx / N, m = idx % N;
    const long row = row0 + rr;
    if (row >= nrows) continue;
    const int q = cart_shift<N>(m);
    cf v = buf[rr * TS + padx<PS>(m)];
    if (INV) {
      v = cscale(v, scale);
      if (smap) v = cconjmul(smap[(row % N) * N + q], v);
      if (accumulate) v = cadd(out[row * N + q], v);
    }
    out[row * N + q] = v;
  }
}

// Column pass over one frame's strip of kCartTX columns. Forward: out = mask * scale * FFT_y(in),
// or with RESID out = that - b and part[block] = the strip's ||out||^2; inverse: out =
// IFFT_y(mask * in).
template <int N, bool INV, bool RESID>
__global__ __launch_bounds__(kBlock) void k_cart_cols(const cf* __restrict__ in, cf* __restrict__ out,
                                                      const uint8_t* __restrict__ mask,
                                                      const cf* __restrict__ twg, const cf* __restrict__ b,
                                                      double* __restrict__ part, float scale) {
  constexpr int TX = kCartTX, P = TX + 1, NS = N / TX;
  constexpr int PT = (N * TX + kBlock - 1) / kBlock;
  __shared__ cf S[N * P];
  __shared__ cf tw[N];
  __shared__ double red[kBlock / 64];
  const int tid = threadIdx.x;
  const long f = blockIdx.x / NS;
  const int c0 = (blockIdx.x % NS) * TX;
  for (int i = tid; i < N; i += kBlock) tw[i] = twg[i];
  const size_t base = (size_t)f * N * N + c0;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * kBlock;
    if (idx < N * TX) {
      const int p = idx / TX, c = idx % TX;
      const size_t o = base + (size_t)p * N + c;
      cf v = in[o];
      if (INV && !mask[o]) v = cf{0.f, 0.f};
      S[cart_shift<N>(p) * P + c] = v;
    }
  }
  lds_sync();
  lds_fft<N, TX / 4, P, 1, true, INV, 0, false, false, true>(S, tw);   // each wave its 4 columns
  lds_sync();
  double q = 0.0;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * kBlock;
    if (idx < N * TX) {
      const int m = idx / TX, c = idx % TX;
      const size_t o = base + (size_t)cart_shift<N>(m) * N + c;
      cf v = S[m * P + c];
      if (!INV) {
        v = mask[o] ? cscale(v, scale) : cf{0.f, 0.f};
        if (RESID) {
          const cf bv = b[o];
          v = cf{v.x - bv.x, v.y - bv.y};
          q += (double)v.x * v.x + (double)v.y * v.y;
        }
      }
      out[o] = v;
    }
  }
  if (RESID) {
    for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o);
    if ((tid & 63) == 0) red[tid >> 6] = q;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) t += red[w];
      part[blockIdx.x] = t;
    }
  }
}

bool cart_supported(int N) {
  switch (N) {
    case 32: case 64: case 128: case 192: case 256: case 320: case 384: case 512: return true;
    default: return false;
  }
}

long cart_part_blocks(int N, int L) { return (long)L * (N / kCartTX); }

namespace {

template <int N>
void fwd_n(const CartOp& op, const cf* img, cf* out, cf* T, const cf* smap, const cf* b, double* part,
           hipStream_t s) {
  const long nrows = (long)op.L * N;
  constexpr int RPB = cart_rpb<N>();
  const unsigned rb = (unsigned)((nrows + RPB - 1) / RPB), cb = (unsigned)cart_part_blocks(N, op.L);
  MRF_LAUNCH("cart_rows_fwd", s, k_cart_rows<N, false><<<rb, kBlock, 0, s>>>(img, T, op.tw, nrows, smap, 0, 1.f));
  if (b) {
    MRF_LAUNCH("cart_cols_fwd", s, k_cart_cols<N, false, true><<<cb, kBlock, 0, s>>>(T, out, op.mask, op.tw, b, part,
                                                                                   1.0f / N));
  } else {
    MRF_LAUNCH("cart_cols_fwd", s, k_cart_cols<N, false, false><<<cb, kBlock, 0, s>>>(T, out, op.mask, op.tw, nullptr,
                                                                                    nullptr, 1.0f / N));
  }
}

template <int N>
void adj_n(const CartOp& op, const cf* ksp, cf* img, cf* T, const cf* smap, int accumulate, hipStream_t s) {
  const long nrows = (long)op.L * N;
  constexpr int RPB = cart_rpb<N>();
  const unsigned rb = (unsigned)((nrows + RPB - 1) / RPB), cb = (unsigned)cart_part_blocks(N, op.L);
  MRF_LAUNCH("cart_cols_adj", s, k_cart_cols<N, true, false><<<cb, kBlock, 0, s>>>(ksp, T, op.mask, op.tw, nullptr,
                                                                                 nullptr, 1.f));
  MRF_LAUNCH("cart_rows_adj", s, k_cart_rows<N, true><<<rb, kBlock, 0, s>>>(T, img, op.tw, nrows, smap, accumulate,
                                                                          1.0f / N));
}

#define MRF_CART_DISPATCH(FN, ...)                                            \
  switch (op.N) {                                                             \
    case 32: FN<32>(__VA_ARGS__); break;                                      \
    case 64: FN<64>(__VA_ARGS__); break;                                      \
    case 128: FN<128>(__VA_ARGS__); break;                                    \
    case 192: FN<192>(__VA_ARGS__); break;                                    \
    case 256: FN<256>(__VA_ARGS__); break;                                    \
    case 320: FN<320>(__VA_ARGS__); break;                                    \
    case 384: FN<384>(__VA_ARGS__); break;                                    \
    case 512: FN<512>(__VA_ARGS__); break;                                    \
    default: return fail(MRF_SHAPE, "cartesian: unsupported image size");     \
  }

}  // namespace

// ksp = M F (S img); T: L N^2 complex of workspace.
mrf_status cart_fwd(const CartOp& op, const cf* img, cf* ksp, cf* T, const cf* smap, hipStream_t s) {
  MRF_CART_DISPATCH(fwd_n, op, img, ksp, T, smap, nullptr, nullptr, s);
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// r = M F (S img) - b and part[0 .. cart_part_blocks) = block partials of ||r||^2.
mrf_status cart_resid(const CartOp& op, const cf* img, const cf* b, cf* r, cf* T, double* part, const cf* smap,
                      hipStream_t s) {
  MRF_CART_DISPATCH(fwd_n, op, img, r, T, smap, b, part, s);
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// img (+)= conj(S) F^H (M ksp).
mrf_status cart_adj(const CartOp& op, const cf* ksp, cf* img, cf* T, const cf* smap, int accumulate, hipStream_t s) {
  MRF_CART_DISPATCH(adj_n, op, ksp, img, T, smap, accumulate, s);
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

}  // namespace mrf
