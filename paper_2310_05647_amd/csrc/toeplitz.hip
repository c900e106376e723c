// Toeplitz normal operator: A^H A of the gradient in eq. (15) applied as a convolution. For frame
// l, (A^H A X)[v] = sum_v' K_l[v - v'] X[v'] with K_l[d] = (1/N^2) sum_j exp(i omega_j . d): the
// centre offsets of A and A^H cancel, so A^H A is a convolution with the point-spread kernel. On
// the 2N grid the linear convolution of the N x N image equals a circular one (no output of the
// N x N window wraps), so
//     A^H A X = crop( IFFT_2N( Khat_l * FFT_2N(pad X) ) ),   Khat_l = FFT_2N(K~_l) / (2N)^2,
// where K~ holds K at (d mod 2N) and zero at the offsets -N that never occur; K~ is Hermitian and
// Khat real. The loop then needs no spreading or interpolation: three passes on the 2N grid
// (the padded row FFTs of the gridded forward transform, a column pass that multiplies by Khat
// between the forward and inverse column FFTs, the cropped inverse row FFTs).
//
// Setup: K~ is the gridded adjoint of all-ones data on a 2N image of the same samples (a plan of
// twice the image side): (1/(2N)) sum_j exp(i omega . (v - N)) = (N/2) K[v - N]. Its 2D FFT is
// taken once, scaled by 1/(2N)^2 and stored as float32, strip-major so that each column-pass
// block reads one contiguous tile: khat[l][strip][ky][c] = Khat_l[ky][strip * kToepTX + c].
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"
#include "fft.hpp"

namespace mrf {
mrf_status rows_fwd_padded(int G, const cf* X, cf* T, const float* dinv, const cf* tw, int nrows, hipStream_t s);
mrf_status rows_adj_cropped(int G, const cf* T, cf* X, const float* dinv, const cf* tw, int nrows, float scale,
                            hipStream_t s);

constexpr int kToepTX = 8;   // grid columns per column-pass block (2 per wave)

// Column pass of the apply: per (frame, strip of kToepTX columns) the N non-zero rows of T
// (centred: row y at (y - N/2) mod G), forward FFT along y, times Khat, inverse FFT, the N rows
// written back in place.
template <int G>
__global__ __launch_bounds__(kBlock) void k_toep_cols(cf* __restrict__ T, const float* __restrict__ khat,
                                                      const cf* __restrict__ twg) {
  constexpr int N = G / 2, TX = kToepTX, P = TX + 1, NS = G / TX;
  constexpr int PT = (N * TX + kBlock - 1) / kBlock;   // T elements per thread
  constexpr int PK = (G * TX + kBlock - 1) / kBlock;   // Khat values per thread
  __shared__ cf S[G * P];
  __shared__ cf tw[G];
  const int tid = threadIdx.x;
  const long f = blockIdx.x / NS;
  const int strip = blockIdx.x % NS, c0 = strip * TX;
  cf* Tf = T + (size_t)f * N * G;
  const float* kh = khat + ((size_t)f * NS + strip) * G * TX;
  cf pre[PT];
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * kBlock;
    if (idx < N * TX) pre[i] = Tf[(size_t)(idx / TX) * G + c0 + idx % TX];
  }
  float kv[PK];
#pragma unroll
  for (int i = 0; i < PK; ++i) {
    const int idx = tid + i * kBlock;
    kv[i] = idx < G * TX ? kh[idx] : 0.f;
  }
  for (int i = tid; i < G; i += kBlock) tw[i] = twg[i];
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * kBlock;
    if (idx < N * TX) {
      int n = idx / TX - N / 2;
      if (n < 0) n += G;
      S[n * P + idx % TX] = pre[i];
    }
  }
  lds_sync();
  // rows [N/2, G - N/2) are the zero padding: the first pass does not read them
  lds_fft<G, TX / 4, P, 1, true, false, 0, true, false, true>(S, tw);
  lds_sync();
#pragma unroll
  for (int i = 0; i < PK; ++i) {
    const int idx = tid + i * kBlock;
    if (idx < G * TX) {
      cf& v = S[(idx / TX) * P + idx % TX];
      v = cscale(v, kv[i]);
    }
  }
  lds_sync();
  // only the N rows of the crop are stored by the last pass
  lds_fft<G, TX / 4, P, 1, true, true, 0, false, true, true>(S, tw);
  lds_sync();
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * kBlock;
    if (idx < N * TX) {
      int n = idx / TX - N / 2;
      if (n < 0) n += G;
      Tf[(size_t)(idx / TX) * G + c0 + idx % TX] = S[n * P + idx % TX];
    }
  }
}

// ---------------------------------------------------------------- setup kernels
__global__ void k_fill_ones(cf* __restrict__ a, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = cf{1.f, 0.f};
}

// K~[l][q] = (2/N) img[l][(q + N) mod G] per axis (img: the adjoint on the 2N image, index v <->
// offset v - N), zero at the offset -N of either axis (q = N).
__global__ void k_psf_embed(const cf* __restrict__ img, cf* __restrict__ Kt, int L, int N) {
  const int G = 2 * N;
  const long total = (long)L * G * G;
  const float sc = 2.0f / (float)N;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long f = i / ((long)G * G);
    const int qy = (int)((i / G) % G), qx = (int)(i % G);
    cf v = {0.f, 0.f};
    if (qy != N && qx != N) {
      const int vy = qy + N < G ? qy + N : qy - N, vx = qx + N < G ? qx + N : qx - N;
      v = cscale(img[(f * G + vy) * G + vx], sc);
    }
    Kt[i] = v;
  }
}

// In-place FFT of every row (length G) of a [rows][G] array.
template <int G>
__global__ __launch_bounds__(kBlock) void k_fft_rows(cf* __restrict__ A, const cf* __restrict__ twg, long nrows) {
  constexpr int RPB = kBlock * 8 / G > 0 ? kBlock * 8 / G : 1;
  constexpr int PS = 3;
  constexpr int TS = padx<PS>(G) + 1;
  __shared__ cf buf[RPB * TS];
  __shared__ cf tw[G];
  const int tid = threadIdx.x;
  for (int i = tid; i < G; i += kBlock) tw[i] = twg[i];
  const long row0 = (long)blockIdx.x * RPB;
  for (int idx = tid; idx < RPB * G; idx += kBlock) {
    const long row = row0 + idx / G;
    buf[(idx / G) * TS + padx<PS>(idx % G)] = row < nrows ? A[row * G + idx % G] : cf{0.f, 0.f};
  }
  lds_sync();
  lds_fft<G, RPB, 1, TS, false, false, PS>(buf, tw);
  for (int idx = tid; idx < RPB * G; idx += kBlock) {
    const long row = row0 + idx / G;
    if (row < nrows) A[row * G + idx % G] = buf[(idx / G) * TS + padx<PS>(idx % G)];
  }
}

// FFT of every column of each frame's G x G array, real part times scale into the strip-major
// khat.
template <int G>
__global__ __launch_bounds__(kBlock) void k_fft_cols_real(const cf* __restrict__ A, float* __restrict__ khat,
                                                          const cf* __restrict__ twg, float scale) {
  constexpr int TX = kToepTX, P = TX + 1, NS = G / TX;
  __shared__ cf S[G * P];
  __shared__ cf tw[G];
  const int tid = threadIdx.x;
  const long f = blockIdx.x / NS;
  const int strip = blockIdx.x % NS, c0 = strip * TX;
  for (int i = tid; i < G; i += kBlock) tw[i] = twg[i];
  const cf* Af = A + (size_t)f * G * G;
  for (int idx = tid; idx < G * TX; idx += kBlock) S[(idx / TX) * P + idx % TX] = Af[(size_t)(idx / TX) * G + c0 + idx % TX];
  lds_sync();
  lds_fft<G, TX / 4, P, 1, true, false, 0, false, false, true>(S, tw);
  lds_sync();
  float* kh = khat + ((size_t)f * NS + strip) * G * TX;
  for (int idx = tid; idx < G * TX; idx += kBlock) kh[idx] = S[(idx / TX) * P + idx % TX].x * scale;
}

namespace {
template <int G>
void apply_g(const cf* X, cf* Y, cf* T, const float* khat, const cf* tw, const float* ones, int L,
             hipStream_t s, mrf_status* st) {
  constexpr int N = G / 2;
  if ((*st = rows_fwd_padded(G, X, T, ones, tw, L * N, s))) return;
  MRF_LAUNCH("toeplitz_cols", s, k_toep_cols<G><<<(unsigned)((long)L * (G / kToepTX)), kBlock, 0, s>>>(T, khat, tw));
  *st = rows_adj_cropped(G, T, Y, ones, tw, L * N, 1.0f, s);
}

template <int G>
void prep_g(cf* Kt, float* khat, const cf* tw, int L, hipStream_t s) {
  constexpr int RPB = kBlock * 8 / G > 0 ? kBlock * 8 / G : 1;
  const long nrows = (long)L * G;
  MRF_LAUNCH("toeplitz_prep", s, k_fft_rows<G><<<(unsigned)((nrows + RPB - 1) / RPB), kBlock, 0, s>>>(Kt, tw, nrows));
  MRF_LAUNCH("toeplitz_prep", s, k_fft_cols_real<G><<<(unsigned)((long)L * (G / kToepTX)), kBlock, 0, s>>>(
                                     Kt, khat, tw, 1.0f / ((float)G * (float)G)));
}

#define MRF_TOEP_DISPATCH(FN, ...)                                              \
  switch (T->G) {                                                               \
    case 32: FN<32>(__VA_ARGS__); break;                                        \
    case 64: FN<64>(__VA_ARGS__); break;                                        \
    case 128: FN<128>(__VA_ARGS__); break;                                      \
    case 256: FN<256>(__VA_ARGS__); break;                                      \
    case 512: FN<512>(__VA_ARGS__); break;                                      \
    default: return fail(MRF_SHAPE, "toeplitz: unsupported image size");       \
  }
}  // namespace

}  // namespace mrf

using namespace mrf;

struct mrf_toeplitz_s {
  int N, G, L;
  float* khat;   // [L][G / kToepTX][G][kToepTX]
  cf* tw;        // [G] exp(-2 pi i k / G)
  float* ones;   // [N] unit deapodisation for the shared row passes
  size_t ws_bytes;
};

namespace {
mrf_status toep_apply(const mrf_toeplitz_s* T, const cf* X, cf* Y, void* ws, hipStream_t s) {
  mrf_status st = MRF_OK;
  MRF_TOEP_DISPATCH(apply_g, X, Y, (cf*)ws, T->khat, T->tw, T->ones, T->L, s, &st);
  if (st) return st;
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}
}  // namespace

namespace mrf {
// for the recon: T (the Toeplitz handle) applied into Y with its own workspace
mrf_status toeplitz_apply(const mrf_toeplitz_s* T, const cf* X, cf* Y, void* ws, hipStream_t s) {
  return toep_apply(T, X, Y, ws, s);
}
size_t toeplitz_ws_bytes(const mrf_toeplitz_s* T) { return T->ws_bytes; }
int toeplitz_n(const mrf_toeplitz_s* T) { return T->N; }
int toeplitz_frames(const mrf_toeplitz_s* T) { return T->L; }
}  // namespace mrf

extern "C" mrf_status mrf_toeplitz_create(const mrf_nufft_desc* d, const float* traj, hipStream_t s,
                                          mrf_toeplitz_t* out) {
  clear_error();
  MRF_REQUIRE(d && traj && out, MRF_INVALID_ARG, "toeplitz_create: null argument");
  *out = nullptr;
  const int N = d->n, G = 2 * N, L = d->nframes;
  MRF_REQUIRE(N == 16 || N == 32 || N == 64 || N == 128 || N == 256, MRF_SHAPE,
              "toeplitz_create: n must be 16, 32, 64, 128 or 256 (the kernel needs a plan of side 2n)");
  MRF_REQUIRE(L >= 1 && d->nsamp >= 1, MRF_INVALID_ARG, "toeplitz_create: nframes, nsamp must be >= 1");
  // the plan of side 2n (grid 4n) that grids the point-spread kernel
  mrf_nufft_desc d2 = *d;
  d2.n = G;
  d2.tile_cols = 0;
  mrf_nufft_plan_t p2 = nullptr;
  mrf_status st = mrf_nufft_plan_create(&d2, traj, s, &p2);
  if (st) return st;
  size_t ws2 = 0;
  mrf_nufft_workspace_size(p2, &ws2);
  const size_t nimg2 = (size_t)L * G * G, nk = (size_t)L * d->nsamp;
  auto* T = new mrf_toeplitz_s{};
  T->N = N; T->G = G; T->L = L;
  T->ws_bytes = (size_t)L * N * G * sizeof(cf);
  void *ws = nullptr, *ones_k = nullptr, *img = nullptr;
  auto cleanup = [&](bool all) {
    hipFree(ws); hipFree(ones_k); hipFree(img);
    mrf_nufft_plan_destroy(p2);
    if (all) {
      hipFree(T->khat); hipFree(T->tw); hipFree(T->ones);
      delete T;
    }
  };
  // ws2 >= L (2N)(4N) complex holds K~ (L (2N)^2 complex) after the adjoint is done with it
  if (hipMalloc(&ws, std::max(ws2, nimg2 * sizeof(cf))) != hipSuccess ||
      hipMalloc(&ones_k, nk * sizeof(cf)) != hipSuccess || hipMalloc(&img, nimg2 * sizeof(cf)) != hipSuccess ||
      hipMalloc(&T->khat, nimg2 * sizeof(float)) != hipSuccess || hipMalloc(&T->tw, G * sizeof(cf)) != hipSuccess ||
      hipMalloc(&T->ones, N * sizeof(float)) != hipSuccess) {
    cleanup(true);
    return fail(MRF_OOM, "toeplitz_create: device allocation failed");
  }
  std::vector<cf> tw(G);
  for (int k = 0; k < G; ++k) tw[k] = cf{(float)std::cos(-2.0 * M_PI * k / G), (float)std::sin(-2.0 * M_PI * k / G)};
  std::vector<float> ones(N, 1.0f);
  hipError_t e = hipMemcpy(T->tw, tw.data(), G * sizeof(cf), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(T->ones, ones.data(), N * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    cleanup(true);
    return fail(MRF_DEVICE, std::string("toeplitz_create: upload: ") + hipGetErrorString(e));
  }
  k_fill_ones<<<1024, 256, 0, s>>>((cf*)ones_k, (long)nk);
  st = mrf_nufft_adj(p2, (const mrf_c64*)ones_k, (mrf_c64*)img, ws, ws2, s);
  if (st == MRF_OK) {
    k_psf_embed<<<4096, 256, 0, s>>>((const cf*)img, (cf*)ws, L, N);
    auto prep = [&]() -> mrf_status {
      MRF_TOEP_DISPATCH(prep_g, (cf*)ws, T->khat, T->tw, L, s);
      MRF_CHECK_LAUNCH();
      return MRF_OK;
    };
    st = prep();
  }
  if (st == MRF_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(MRF_DEVICE, std::string("toeplitz_create: ") + hipGetErrorString(e));
  }
  if (st != MRF_OK) {
    cleanup(true);
    return st;
  }
  cleanup(false);
  *out = T;
  return MRF_OK;
}

extern "C" mrf_status mrf_toeplitz_destroy(mrf_toeplitz_t T) {
  clear_error();
  if (!T) return MRF_OK;
  hipFree(T->khat); hipFree(T->tw); hipFree(T->ones);
  delete T;
  return MRF_OK;
}

extern "C" mrf_status mrf_toeplitz_workspace_size(mrf_toeplitz_t T, size_t* bytes) {
  clear_error();
  MRF_REQUIRE(T && bytes, MRF_INVALID_ARG, "toeplitz_workspace_size: null argument");
  *bytes = T->ws_bytes;
  return MRF_OK;
}

extern "C" mrf_status mrf_toeplitz_normal(mrf_toeplitz_t T, const mrf_c64* X, mrf_c64* Y, void* ws, size_t ws_bytes,
                                          hipStream_t s) {
  clear_error();
  MRF_REQUIRE(T && X && Y, MRF_INVALID_ARG, "toeplitz_normal: null argument");
  MRF_REQUIRE(ws && ws_bytes >= T->ws_bytes, MRF_WORKSPACE, "toeplitz_normal: workspace missing or too small");
  return toep_apply(T, (const cf*)X, (cf*)Y, ws, s);
}
