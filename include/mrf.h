/* libmrf: MI355X (gfx950) hot path of the MS-LLR MR-fingerprinting reconstruction
 * (Li, Ji, Hu: "Exploiting Manifold Structured Data Priors for Improved MR Fingerprinting
 * Reconstruction", arXiv 2310.05647).
 *
 * Conventions shared by every call:
 *  - Arrays are caller-owned DEVICE memory unless a comment says "host". Complex data
 *    are interleaved (re, im) float32 pairs, the layout of torch.complex64.
 *  - Image series are frame-major: X[l][y][x], l < L, y, x < N (x fastest).
 *  - Opaque handles are library-owned; create/destroy them explicitly. A handle must not
 *    be used from two host threads at once.
 *  - Every call returns an mrf_status. Arguments are checked on the host before anything
 *    is enqueued; on error nothing is enqueued and mrf_last_error() describes why.
 *  - Work is enqueued on the caller's stream and is asynchronous unless stated otherwise.
 *    Faults inside kernels surface at the next synchronising call.
 */
#ifndef MRF_H
#define MRF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mrf_status {
  MRF_OK = 0,
  MRF_INVALID_ARG = 1,   /* null pointer, non-positive size, bad enum value        */
  MRF_SHAPE = 2,         /* a size outside what the kernels support                 */
  MRF_WORKSPACE = 3,     /* workspace missing or smaller than the queried size      */
  MRF_DEVICE = 4,        /* a HIP runtime call or kernel launch failed              */
  MRF_OOM = 5,           /* device allocation of a handle's tables failed           */
  MRF_NONFINITE = 6,     /* a cost value became NaN or Inf                          */
  MRF_NOT_SUPPORTED = 7  /* a valid request this build does not implement           */
} mrf_status;

typedef struct mrf_c64 {
  float re, im;
} mrf_c64;

/* Human-readable name of a status code (static string). */
const char* mrf_status_string(mrf_status st);
/* Message of the last failing call on this host thread ("" if none). */
const char* mrf_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int mrf_version(void);

/* Per-kernel timing for benchmarks. While enabled, every kernel launch of the library is
 * bracketed by two HIP events recorded on the stream the kernel is launched on. */
mrf_status mrf_timing_enable(int on);
/* Synchronises the recorded events and writes one line per kernel name into buf (host):
 * "<name> <launches> <total_ms> <min_ms> <max_ms>\n", truncated to buf_len - 1 bytes.
 * Clears the records. */
mrf_status mrf_timing_report(char* buf, size_t buf_len);

/* ====================================================================================
 * NUFFT pair: the single-coil acquisition operator A = F_u of eq. (1) and its adjoint A^H,
 * used in the gradient step eq. (15) and for X^0 = A^H b (Algorithm 1).
 *
 * Definition: b_l[j] = (1/N) sum_{y,x} X_l[y,x] exp(-i(wx (x - N/2) + wy (y - N/2))), with
 * (wx, wy) = traj[l][j] in rad/pixel, in [-pi, pi). Computed by Kaiser-Bessel gridding on a
 * 2N x 2N grid with width 6 (beta of Beatty et al. 2005), deapodisation by the kernel's
 * Fourier transform, taps floor(u)-2 .. floor(u)+3 with u = w * 2N / (2 pi). mrf_nufft_adj
 * is the exact adjoint of mrf_nufft_fwd (same real weights).
 * ==================================================================================== */
typedef struct mrf_nufft_plan_s* mrf_nufft_plan_t;

typedef struct mrf_nufft_desc {
  int n;          /* image side N; a power of two, 16 <= N <= 512                      */
  int nframes;    /* L >= 1                                                            */
  int nsamp;      /* Ns >= 1 samples per frame                                         */
  int kb_width;   /* must be 6                                                         */
  int oversamp;   /* must be 2 (grid side G = 2N)                                      */
  int tile_cols;  /* grid columns per spread/interpolation strip: 0 = default (8;
                     16 when G = 32); otherwise 8, 16, or 32 (G <= 128), at most G/2    */
} mrf_nufft_desc;

/* Builds the plan for a fixed trajectory: traj is device float32 [L][Ns][2] (wx, wy).
 * Sorts the samples into grid tiles (with halo duplication), precomputes the Kaiser-Bessel
 * tap weights and the deapodisation. Synchronises `stream`. Tables are device memory owned
 * by the plan (about 64 bytes per sample and tile it touches). */
mrf_status mrf_nufft_plan_create(const mrf_nufft_desc* desc, const float* traj,
                                 hipStream_t stream, mrf_nufft_plan_t* out);
mrf_status mrf_nufft_plan_destroy(mrf_nufft_plan_t plan);
/* Bytes of caller-provided device workspace that mrf_nufft_fwd / mrf_nufft_adj need. */
mrf_status mrf_nufft_workspace_size(mrf_nufft_plan_t plan, size_t* bytes);
/* ksp [L][Ns] = A img, img [L][N][N]. ws: device workspace of at least the queried size. */
mrf_status mrf_nufft_fwd(mrf_nufft_plan_t plan, const mrf_c64* img, mrf_c64* ksp,
                         void* ws, size_t ws_bytes, hipStream_t stream);
/* img [L][N][N] = A^H ksp, ksp [L][Ns]. */
mrf_status mrf_nufft_adj(mrf_nufft_plan_t plan, const mrf_c64* ksp, mrf_c64* img,
                         void* ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MRF_H */
