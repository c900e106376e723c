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
  MRF_NOT_SUPPORTED = 7  /* a valid request the library does not implement          */
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
/* "sources-sha256=<hex> built=<UTC time> arch=gfx950": the SHA-256 over the library's sources
 * (csrc/ and include/, in name order) as the build step saw them, and when it ran. Static string. */
const char* mrf_build_info(void);

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
  int n;          /* image side N: 16, 32, 64, 128, 192, 256, 320 or 512 (G = 2N)      */
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
/* Autotuner: for the trajectory traj (as in mrf_nufft_plan_create) times reps forward + adjoint
 * pairs on a pseudo-random image for each strip width tile_cols in {8, 16, 32} that the grid
 * allows, writes their mean pair times (ms; -1 where not allowed) to pair_ms [3] (optional) and
 * the fastest width to best_tile_cols (use it as desc.tile_cols). Allocates and frees its own
 * buffers; synchronises. */
mrf_status mrf_nufft_autotune(const mrf_nufft_desc* desc, const float* traj, int reps, int* best_tile_cols,
                              float* pair_ms, hipStream_t stream);
/* lambda_max(A^H A) estimated by `iters` power iterations from a deterministic start vector
 * (seeded hash), written to *lam (host). Setup call: allocates temporary device memory and
 * synchronises. Algorithm 1's step-size rule takes this bound (see mrf_recon_params.lamA). */
mrf_status mrf_nufft_opnorm(mrf_nufft_plan_t plan, int iters, unsigned seed, double* lam, hipStream_t stream);

/* Pseudo-radial Cartesian sampling (Sec. IV, the third sampling pattern): a plan whose operator is
 * A_l X_l = M_l (F X_l), F the unitary centred 2D DFT (the definition above with every frequency
 * on the integer grid, w = 2 pi k / N: k-space point [ky + n/2][kx + n/2] holds frequency
 * (kx, ky)) and M_l the 0/1 mask of frame l. mask: uint8 [nframes][n][n] (host or device;
 * copied into the plan). The plan serves every call that takes an mrf_nufft_plan_t (fwd, adj,
 * the multi-coil calls, opnorm, mrf_recon_create) with Ns = n * n: ksp is the dense masked
 * k-space [L][n][n], zero where the mask is; the adjoint applies the mask to its input first.
 * n: 32, 64, 128, 192, 256, 320, 384 or 512. Workspace: L n^2 complex64. Synchronises `stream`.
 * mrf_nufft_autotune does not apply. MRF_SHAPE for an unsupported n, MRF_OOM. */
mrf_status mrf_cart_plan_create(int n, int nframes, const uint8_t* mask, hipStream_t stream,
                                mrf_nufft_plan_t* out);

/* Toeplitz normal operator for the gradient of eq. (15): A^H A X as a convolution of each frame
 * with its point-spread kernel K_l[d] = (1/N^2) sum_j exp(i omega_j . d) (the centre offsets of A
 * and A^H cancel), done as a circular convolution on the 2N x 2N grid: the padded row FFTs, a
 * column pass multiplying the 2D spectrum by the real kernel spectrum, the cropped inverse row
 * FFTs. No spreading or interpolation runs per application.
 * mrf_toeplitz_create: desc and traj as for mrf_nufft_plan_create (n: 16, 32, 64, 128 or 256); the
 *   kernel is the gridded adjoint of unit data on a 2n image of the same samples (a temporary plan
 *   of side 2n), its spectrum stored as float32 [L][2n][2n] (4 L (2n)^2 bytes, owned by the
 *   handle). Setup call: allocates temporaries of about L (2n)^2 24 bytes, synchronises.
 * mrf_toeplitz_normal: Y [L][n][n] = A^H A X, X [L][n][n]; ws of mrf_toeplitz_workspace_size
 *   (8 L n 2n bytes). Asynchronous. X and Y may not alias.
 * Within the KB error of the gridded pair (mrf_nufft_adj of mrf_nufft_fwd). MRF_SHAPE for an
 * unsupported n, MRF_WORKSPACE for a short workspace, MRF_OOM. */
typedef struct mrf_toeplitz_s* mrf_toeplitz_t;
mrf_status mrf_toeplitz_create(const mrf_nufft_desc* desc, const float* traj, hipStream_t stream,
                               mrf_toeplitz_t* out);
mrf_status mrf_toeplitz_destroy(mrf_toeplitz_t t);
mrf_status mrf_toeplitz_workspace_size(mrf_toeplitz_t t, size_t* bytes);
mrf_status mrf_toeplitz_normal(mrf_toeplitz_t t, const mrf_c64* X, mrf_c64* Y, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/* FISP signal model (eqs. (2)-(3)) by the extended phase graph, on the device: the dictionary
 * atoms d_m = B(eta_m; theta) with PD = 1 and off-grid training signals. States F+_k, F-_k, Z_k,
 * k < n_states; an ideal inversion and one TR of recovery, then per frame l an RF rotation about
 * x by fa_deg[l] * b1[m] degrees, the signal F+_0 exp(-TE/T2), relaxation over tr_ms[l] and one
 * dephasing shift (orders >= n_states dropped).
 * mrf_epg_fisp: t1, t2 [n_atoms] (ms), b1 [n_atoms] or NULL (1), fa_deg, tr_ms [n_frames] (all
 *   device float32); out [n_atoms][n_frames] complex64 (device, caller-owned; unnormalised: pass
 *   it to mrf_dict_create as is). n_states: 8, 16, 24 or 32 (MRF_SHAPE otherwise). FP32,
 *   asynchronous. MRF_INVALID_ARG for null pointers, sizes < 1 or te_ms < 0.
 * mrf_epg_random_params: params [n][3] (device) = (T1, T2, B1) drawn by Philox4x32-10 (counter
 *   (i, 0x45504731, 0, 0), key = seed): T1 log-uniform on [t1_lo, t1_hi], T2 log-uniform on
 *   [t2_lo, min(t2_hi, T1)] (so T2 <= T1, the rule of the paper's dictionary), B1 uniform on
 *   [b1_lo, b1_hi]. Needs 0 < t2_lo <= t1_lo <= t1_hi, t2_lo <= t2_hi, b1_lo <= b1_hi.
 * mrf_epg_params_to_columns: cols [3][n] (T1 row, T2 row, B1 row) from params [n][3], the inputs
 *   of mrf_epg_fisp. */
mrf_status mrf_epg_fisp(int n_atoms, int n_frames, int n_states, const float* t1, const float* t2, const float* b1,
                        const float* fa_deg, const float* tr_ms, float te_ms, mrf_c64* out, hipStream_t stream);
mrf_status mrf_epg_random_params(int n, uint64_t seed, float t1_lo, float t1_hi, float t2_lo, float t2_hi,
                                 float b1_lo, float b1_hi, float* params, hipStream_t stream);
mrf_status mrf_epg_params_to_columns(int n, const float* params, float* cols, hipStream_t stream);

/* Multi-coil acquisition (Sec. II, eq. (1)): the forward operator is F_u C, where C multiplies
 * every frame by each coil's sensitivity map and F_u is the single-coil operator above.
 *   smaps  device complex64 [ncoils][N][N], one map per coil, shared by all frames; caller-owned,
 *          read during the call only.
 *   ksp    [ncoils][L][Ns]: coil c's series at ksp + c L Ns.
 * mrf_nufft_fwd_mc : ksp_c = A (S_c img) for every coil.
 * mrf_nufft_adj_mc : img = sum_c conj(S_c) A^H ksp_c, coils summed in index order (overwrites
 *                    img; deterministic run to run).
 * Same workspace as the single-coil calls (coils run one after another on `stream`; the cost is
 * ncoils single-coil transforms). Errors: MRF_INVALID_ARG for null pointers or ncoils < 1,
 * MRF_WORKSPACE for a missing or short workspace. */
mrf_status mrf_nufft_fwd_mc(mrf_nufft_plan_t plan, const mrf_c64* smaps, int ncoils, const mrf_c64* img,
                            mrf_c64* ksp, void* ws, size_t ws_bytes, hipStream_t stream);
mrf_status mrf_nufft_adj_mc(mrf_nufft_plan_t plan, const mrf_c64* smaps, int ncoils, const mrf_c64* ksp,
                            mrf_c64* img, void* ws, size_t ws_bytes, hipStream_t stream);
/* lambda_max((F_u C)^H F_u C) by power iteration, as mrf_nufft_opnorm (smaps null: single coil). */
mrf_status mrf_nufft_opnorm_mc(mrf_nufft_plan_t plan, const mrf_c64* smaps, int ncoils, int iters, unsigned seed,
                               double* lam, hipStream_t stream);


/* ====================================================================================
 * Patch graph on the parameter manifold (Sec. III-A): eq. (8) weights, eq. (10) Laplacian,
 * and its use in the manifold term Tr(Q(X) L Q(X)^H) of eq. (9) / gradient of eq. (15).
 * Patches are p x p with stride s (the paper's 11/5; the stride is floor(p/2)), origins
 * (a s, b s), numbered in raster order; p % s == 0 and (n - p) % s == 0 are required.
 * The graph keeps the K nearest patches by squared distance of the patch features (self
 * excluded, ties to the lower index), symmetrised by W = max(W, W^T); the features are the
 * (T1, T2, PD) map patches with every channel divided by its maximum over the map.
 * ==================================================================================== */
typedef struct mrf_graph_s* mrf_graph_t;

/* Allocates a graph for n x n maps with p x p patches (p <= 8) at stride s, at most k_max
 * neighbours (k_max <= 16) and Laplacian quadratic forms over at most max_frames frames. The
 * patch count must be in [2, 8192] (a dense Np x Np weight buffer is part of the handle). */
mrf_status mrf_graph_create(int n, int p, int s, int k_max, int max_frames, mrf_graph_t* out);
mrf_status mrf_graph_destroy(mrf_graph_t g);
/* Builds the K-NN graph Laplacian from maps [3][n][n] (T1, T2, PD; device float32).
 * sigma2 > 0 fixes sigma^2 of eq. (8); sigma2 <= 0 takes the lower median of the positive
 * directed K-NN squared distances (1 when there are none). Asynchronous. */
mrf_status mrf_knn_laplacian(mrf_graph_t g, const float* maps, int K, float sigma2, hipStream_t stream);
/* Synchronises `stream` and reports the CSR of L (rows ascending, columns ascending, the
 * diagonal D_ii included; device pointers owned by the graph), sigma^2 and max(L) (the
 * largest entry of L, i.e. the largest degree, used by Algorithm 1's lambda1 schedule).
 * Any output pointer may be NULL. */
mrf_status mrf_graph_info(mrf_graph_t g, int* np, int* nnz, const int** rowptr, const int** col,
                          const float** val, double* sigma2, double* lmax, hipStream_t stream);
/* Y = Q*(Q(X) L) for X, Y [L][n][n] (must not alias). Asynchronous. */
mrf_status mrf_laplacian_apply(mrf_graph_t g, const mrf_c64* X, mrf_c64* Y, int L, hipStream_t stream);
/* out (device double) = Re<X, Q*(Q(X) L)> = Tr(Q(X) L Q(X)^H), X [L][n][n], L <= max_frames. */
mrf_status mrf_laplacian_quad(mrf_graph_t g, const mrf_c64* X, int L, double* out, hipStream_t stream);

/* ====================================================================================
 * Locally low-rank step (Sec. III-C): per patch, singular value thresholding of the p^2 x L
 * Casorati matrix Q_{q_i}(X) (eq. (22), threshold tau = 1/beta), keeping at most rank_cap
 * values, then overlap-add Q*(P') (the term of eq. (23)). Computed from the patch Gram on
 * MFMA (FP32) and its eigen-decomposition in FP64. p must be 2, 3, 4 or 8 and n % 16 == 0.
 * ==================================================================================== */
mrf_status mrf_llr_workspace_size(int n, int L, int p, int s, int rank_cap, size_t* bytes);
/* QtP [L][n][n] = Q*(P'), nuc_norm (device double) = sum_i ||Q_{q_i}(X)||_* over all
 * singular values (eq. (13)). X [L][n][n]. Asynchronous. */
mrf_status mrf_llr_prox(const mrf_c64* X, mrf_c64* QtP, int n, int L, int p, int s, float tau, int rank_cap,
                        double* nuc_norm, void* ws, size_t ws_bytes, hipStream_t stream);

/* The X update of eq. (23) following the SVT of eq. (22):
 *   Xout = (Z + kappa Q*(P')) / (1 + kappa c(v)),  P' = SVT_tau(Q_{q_i}(X)) per patch as in
 *   mrf_llr_prox, kappa = mu lambda2 beta, c(v) the number of patches covering pixel v
 * (eq. (23) divides by the scalar 1 + kappa, exact when patches do not overlap; the per-pixel
 * c(v) makes it the exact minimiser of eq. (21) for overlapping patches). Z [L][n][n] is given
 * either in full (beta_coef = NULL) or, for 8 x 8 patches at stride 4, as the subspace
 * expansion Z = beta_coef V^H of eq. (17) (Z = NULL; beta_coef [n*n][r] voxel-major, V [L][r],
 * 1 <= r <= 16), formed inside the update's tiles and never stored. Xout must not alias X or Z.
 * ws: at least mrf_llr_xupdate_workspace_size bytes. Asynchronous. */
mrf_status mrf_llr_xupdate_workspace_size(int n, int L, int p, int s, int rank_cap, size_t* bytes);
mrf_status mrf_llr_xupdate(const mrf_c64* X, const mrf_c64* Z, const mrf_c64* beta_coef, const mrf_c64* V, int r,
                           int n, int L, int p, int s, float tau, int rank_cap, double kappa, mrf_c64* Xout, void* ws,
                           size_t ws_bytes, hipStream_t stream);

/* ====================================================================================
 * Temporal subspace (Sec. III-B, eq. (17)): P_S(X) = X V V^H for every voxel's time course,
 * with V [L][r] an orthonormal basis approximated from the dictionary (an input, as P_S is
 * among Algorithm 1's predefined inputs). r <= 16. X is frame-major [L][Nv].
 * ==================================================================================== */
mrf_status mrf_subspace_coeffs_workspace_size(int L, int Nv, int r, size_t* bytes);
/* alpha [Nv][r] (voxel-major) = X V. */
mrf_status mrf_subspace_coeffs(const mrf_c64* X, const mrf_c64* V, int L, int Nv, int r, mrf_c64* alpha,
                               void* ws, size_t ws_bytes, hipStream_t stream);
/* For callers that cannot allocate device memory or take a workspace (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): mrf_subspace_coeffs with its
 * partial sums (frame chunks x r x Nv complex values) in a library-owned static device array of
 * 16 MiB per GPU, held until the process ends (enough for Nv = 65 536, r = 10 at any L). Same
 * kernels and result as mrf_subspace_coeffs. MRF_WORKSPACE if the partial sums would exceed
 * 16 MiB. Allocates nothing: no hipMalloc, hipFree or allocating library routine (the first call
 * on a device looks up the array's device address). Every call on one GPU shares the array:
 * calls that overlap on one GPU (several streams or host threads) race, so the caller must order
 * them. Asynchronous. */
mrf_status mrf_subspace_coeffs_noalloc(const mrf_c64* X, const mrf_c64* V, int L, int Nv, int r, mrf_c64* alpha,
                                       hipStream_t stream);
/* Z [L][Nv] = U V V^H; ws needs the coeffs workspace plus Nv * r * 8 bytes. */
mrf_status mrf_subspace_project(const mrf_c64* U, const mrf_c64* V, int L, int Nv, int r, mrf_c64* Z,
                                void* ws, size_t ws_bytes, hipStream_t stream);

/* ====================================================================================
 * Dictionary and pattern matching Phi_D (Sec. II-B, eqs. (3)-(5)).
 * k = argmax_m |<d_m, x>| / ||d_m|| (ties to the lowest m), eta = LUT[k],
 * rho = max(Re<d_k, x> / ||d_k||^2, 0), with <d, x> = sum_l conj(d_l) x_l. (Eq. (5) prints
 * ||d_k||^2 in the arg-max denominator; the arg-max here uses ||d_k||, which coincides with it
 * for unit-norm atoms.)
 * ==================================================================================== */
typedef struct mrf_dict_s* mrf_dict_t;

/* atoms [M][L] complex (PD = 1 atoms, device), lut [M][nparam] float32 (device), V [L][r]
 * or NULL. Keeps the atom norms, the unit-norm atoms (FP32, and BF16 / FP8 copies for the
 * low-precision full-length match) and, with V, the projected unit atoms d_m V / ||d_m|| in MFMA
 * operand order. Synchronises `stream`. 2 <= nparam <= 8, r <= 10. */
mrf_status mrf_dict_create(const mrf_c64* atoms, const float* lut, int M, int L, int nparam, const mrf_c64* V,
                           int r, hipStream_t stream, mrf_dict_t* out);
mrf_status mrf_dict_destroy(mrf_dict_t d);
/* Subspace match of alpha [Nv][r] (= x V per voxel) against d_m V, normalised by ||d_m||:
 * idx [Nv] int32, and optionally rho [Nv], score [Nv] (= |<d_m V, alpha>| / ||d_m||),
 * params [Nv][nparam] (LUT rows). FP32 on MFMA. Asynchronous. */
mrf_status mrf_dict_match_subspace(mrf_dict_t d, const mrf_c64* alpha, int Nv, int32_t* idx, float* rho,
                                   float* score, float* params, hipStream_t stream);

/* Full-length match modes (eq. (5) on length-L fingerprints). Every mode ranks all M atoms by
 * |<d_m, x>| / ||d_m|| computed on MFMA in the stated precision (FP32 accumulation), keeps the
 * four best (ties to the lower index) and re-ranks those four exactly in FP32 from the FP32
 * unit-norm atoms; idx / score / rho / params come from the re-rank.
 *   MRF_MATCH_FP32          scores from FP32 atoms and fingerprints (v_mfma_f32_16x16x4f32)
 *   MRF_MATCH_BF16_RERANK4  atoms and fingerprints rounded to BF16 (v_mfma_f32_16x16x32_bf16)
 *   MRF_MATCH_FP8_RERANK4   OCP E4M3 with one scale per row (max |component| -> 448), FP8 MFMA
 *   MRF_MATCH_BF16X3_RERANK split BF16 (hi + lo parts of atoms and fingerprints), three BF16 MFMA
 *                           products per score: 3x the BF16 work at close to FP32 scores
 *   MRF_MATCH_LEARNED       (C4) the MLP estimate with the residual gate; see mrf_mlp_*      */
typedef enum mrf_match_mode {
  MRF_MATCH_FP32 = 0,
  MRF_MATCH_BF16_RERANK4 = 1,
  MRF_MATCH_FP8_RERANK4 = 2,
  MRF_MATCH_LEARNED = 3,
  MRF_MATCH_SUBSPACE = 4,  /* the subspace match of mrf_dict_match_subspace (only as a final match of mrf_recon) */
  MRF_MATCH_BF16X3_RERANK = 5  /* split BF16: each value as hi + lo BF16 parts, scores from the
                                  three products hi hi + hi lo + lo hi (about 16 mantissa bits) */
} mrf_match_mode;

/* Workspace bytes of mrf_dict_match for Nv fingerprints (FP32 / BF16 / FP8 modes). */
mrf_status mrf_dict_match_workspace_size(mrf_dict_t d, int Nv, mrf_match_mode mode, size_t* bytes);
/* Full-length match of fp [Nv][L] (voxel-major, complex, device; L = the dictionary's length):
 * idx [Nv] int32 (required); rho [Nv], score [Nv], params [Nv][nparam] and cand [Nv][4] (the
 * candidates that entered the re-rank, best first by low-precision score; -1 where fewer than
 * four atoms exist) are optional (NULL). The caller owns all arrays and the workspace.
 * Asynchronous; MRF_NOT_SUPPORTED for MRF_MATCH_LEARNED (use mrf_mlp_match). */
mrf_status mrf_dict_match(mrf_dict_t d, const mrf_c64* fp, int Nv, mrf_match_mode mode, int32_t* idx, float* rho,
                          float* score, float* params, int32_t* cand, void* ws, size_t ws_bytes, hipStream_t stream);
/* mrf_dict_match with the re-rank depth chosen: the `depth` (1..32) best candidates by the
 * mode's scores (each of the 8 atom groups keeps its best 8; the depth best of those 64 are taken,
 * ties to the lower index) are re-ranked exactly in FP32; cand [Nv][depth] (optional). A deeper
 * re-rank recovers the FP32 result where low-precision scores reorder near neighbours of a dense
 * dictionary. mrf_dict_match is depth 4. Same workspace. */
mrf_status mrf_dict_match_depth(mrf_dict_t d, const mrf_c64* fp, int Nv, mrf_match_mode mode, int depth, int32_t* idx,
                                float* rho, float* score, float* params, int32_t* cand, void* ws, size_t ws_bytes,
                                hipStream_t stream);
/* Y [Nv][L] = X [L][Nv] (frame-major image series to voxel-major fingerprints). Asynchronous. */
mrf_status mrf_frames_to_voxels(const mrf_c64* X, int L, int Nv, mrf_c64* Y, hipStream_t stream);

/* ====================================================================================
 * Learned matching (the library's own addition beside eq. (5); the paper cites learned
 * signal-to-parameter mappings as related work, Sec. I). An MLP maps the features of the
 * subspace coefficients alpha = x V (r complex values, normalised, phase-rotated so alpha_0 is
 * real >= 0: 2 r reals) to the standardised (log T1, log T2); ReLU hidden layers.
 * Training batches are drawn on the device: sample i of step s uses Philox4x32-10 with key
 * `seed` and counter (i, s, c, 0) for the atom, the phase, the SNR in [snr_lo, snr_hi] dB and the
 * Box-Muller noise (variance 10^(-SNR/10) / L per coefficient) added to d_m V / ||d_m||. Loss:
 * mean squared error; Adam with bias correction; optional cosine decay of lr over total_steps.
 * GEMMs on MFMA in FP32 or BF16 (operands rounded to nearest even), FP32 accumulation and
 * FP32 master weights. Parameters are one flat FP32 array [W1 b1 W2 b2 ...], W_l [out][in].
 * The gate: k* = the grid atom nearest to the prediction in Euclidean distance on (log T1,
 * log T2), among the grid's atoms (ties to the lower index); residual =
 * 1 - |<d_k* V / ||d_k*||, alpha / ||alpha||>|; voxels with residual > theta take the exhaustive
 * subspace match (mrf_dict_match_subspace) instead.
 * ==================================================================================== */
typedef struct mrf_mlp_s* mrf_mlp_t;

typedef struct mrf_mlp_train_cfg {
  int batch;          /* samples per step                                                  */
  int steps;          /* steps run by this call                                            */
  int first_step;     /* step index of the first one (the counter of the batch generator)   */
  int total_steps;    /* length of the cosine schedule (<= 0: first_step + steps)           */
  float lr, beta1, beta2, eps;
  int cosine;         /* 1: lr_s = lr (1 + cos(pi s / total_steps)) / 2; 0: constant lr      */
  float snr_lo, snr_hi;
  uint64_t seed;
  int bf16;           /* 1: BF16 GEMM operands, 0: FP32                                     */
} mrf_mlp_train_cfg;

/* n_in = 2 r inputs, n_hidden_layers layers of `hidden` units, n_out = 2 outputs; weights
 * He-normal from Philox (key seed, counter (index, layer, 0x48e, 0)), biases 0. Synchronises. */
mrf_status mrf_mlp_create(int n_in, int hidden, int n_hidden_layers, int n_out, uint64_t seed, hipStream_t stream,
                          mrf_mlp_t* out);
mrf_status mrf_mlp_destroy(mrf_mlp_t mlp);
mrf_status mrf_mlp_param_count(mrf_mlp_t mlp, size_t* n);
/* Device pointers to the library-owned flat parameter and gradient arrays (FP32, param_count
 * values each); the caller may read or overwrite them between calls on the same stream. */
mrf_status mrf_mlp_params(mrf_mlp_t mlp, float** params, float** grads);
mrf_status mrf_mlp_reset_optimizer(mrf_mlp_t mlp, hipStream_t stream);
/* The (T1, T2) grid of the gate: n1 T1 values log_t1_0 + i dlog_t1, n2 T2 values likewise;
 * grid_index [n1][n2] (device int32) the atom of each point or -1. Every T1 row must hold an
 * atom, and a row's atoms must occupy T2 indices 0 .. (its largest) without gaps (the T2 <= T1
 * rule of the dictionary gives this); otherwise MRF_INVALID_ARG. mrf_mlp_match returns MRF_SHAPE
 * if the grid names an atom index >= the dictionary's M. Synchronises. */
mrf_status mrf_mlp_set_grid(mrf_mlp_t mlp, int n1, double log_t1_0, double dlog_t1, int n2, double log_t2_0,
                            double dlog_t2, const int32_t* grid_index, hipStream_t stream);
/* Mean and standard deviation of log T1, log T2 over the dictionary (the target scaling);
 * stats_host [4] = (mean1, mean2, std1, std2) if not NULL (synchronises then). */
mrf_status mrf_mlp_target_stats(mrf_mlp_t mlp, mrf_dict_t d, double* stats_host, hipStream_t stream);
mrf_status mrf_mlp_train_workspace_size(mrf_mlp_t mlp, int batch, size_t* bytes);
/* The network's state: parameters, Adam moments and step count, target scaling and the gate's
 * grid. mrf_mlp_state_bytes gives the size; save writes it to buf (host or device memory) and
 * synchronises; load restores it into a network of the same architecture (MRF_SHAPE otherwise),
 * so that inference, and training continued from it, give what the saved network gives. */
mrf_status mrf_mlp_state_bytes(mrf_mlp_t mlp, size_t* bytes);
mrf_status mrf_mlp_save(mrf_mlp_t mlp, void* buf, size_t bytes, hipStream_t stream);
mrf_status mrf_mlp_load(mrf_mlp_t mlp, const void* buf, size_t bytes, hipStream_t stream);
/* One synthetic batch: z [batch][n_in], t [batch][2] (standardised targets), m [batch] or NULL. */
mrf_status mrf_mlp_synth(mrf_mlp_t mlp, mrf_dict_t d, uint64_t seed, int step, int batch, float snr_lo, float snr_hi,
                         float* z, float* t, int32_t* m, hipStream_t stream);
/* y [batch][2] = network(z [batch][n_in]); workspace of mrf_mlp_train_workspace_size(batch). */
mrf_status mrf_mlp_forward(mrf_mlp_t mlp, const float* z, int batch, int bf16, float* y, void* ws, size_t ws_bytes,
                           hipStream_t stream);
/* Loss (device float, may be NULL) and gradients (into the library's gradient array) of a batch. */
mrf_status mrf_mlp_grads(mrf_mlp_t mlp, const float* z, const float* t, int batch, int bf16, float* loss, void* ws,
                         size_t ws_bytes, hipStream_t stream);
/* One Adam update of the parameters from the current gradients. */
mrf_status mrf_mlp_adam_step(mrf_mlp_t mlp, float lr, float beta1, float beta2, float eps, hipStream_t stream);
/* cfg->steps steps of synthesis, forward, backward and Adam; losses [steps] (device) or NULL. */
mrf_status mrf_mlp_train(mrf_mlp_t mlp, mrf_dict_t d, const mrf_mlp_train_cfg* cfg, float* losses, void* ws,
                         size_t ws_bytes, hipStream_t stream);
mrf_status mrf_mlp_match_workspace_size(mrf_mlp_t mlp, int Nv, size_t* bytes);
/* Learned match of alpha [Nv][r]: idx [Nv] (k*, or the exhaustive match's atom where gated out),
 * t12 [Nv][2] (the network's T1, T2, or the exhaustive match's LUT values), rho [Nv], resid [Nv],
 * fallback [Nv] (1 where gated out) optional; n_fallback (host) optional. Synchronises once
 * (the fallback count). */
mrf_status mrf_mlp_match(mrf_mlp_t mlp, mrf_dict_t d, const mrf_c64* alpha, int Nv, int bf16, float theta, int32_t* idx,
                         float* t12, float* rho, float* resid, int32_t* fallback, int* n_fallback, void* ws,
                         size_t ws_bytes, hipStream_t stream);

/* ====================================================================================
 * Algorithm 1: the MS-LLR reconstruction (Sec. III-C, III-D), run on the device.
 *   X^0 = A^H b (or a given X0), M^0 = Phi_D(X^0), L^0 = mrf_knn_laplacian(M^0),
 *   lambda1 = lambda1^0 max(L); per iteration the gradient step of eq. (15) with the
 *   projection P_S (eq. (17)), the SVT of eq. (22) on Q(X^n), the X update of eq. (23) divided
 *   per pixel by 1 + mu lam2 beta c(v) (c = patch coverage), the cost of Algorithm 1 and its
 *   stopping rule cost(n-1)/cost(n) - 1 < tol; then M, L and lambda1 are updated.
 *   Step size mu = min(mu0, 1 / (lamA + 2 c_max lambda1 max(L))) when lamA > 0, else mu0.
 * The matching inside the loop and at the end is the subspace match (mrf_dict_match_subspace).
 * ==================================================================================== */
typedef struct mrf_recon_params {
  int p, s;          /* patch side and stride (p % s == 0, (n - p) % s == 0; p in {2, 3, 4, 8})   */
  int K;             /* graph neighbours                                                          */
  int rank_cap;      /* at most this many singular values kept per patch (1..16)                   */
  float lam1_0;      /* lambda1^0 of the schedule lambda1 = lambda1^0 max(L)                       */
  float lam2;        /* lambda2                                                                   */
  float beta;        /* penalty beta; SVT threshold 1/beta                                        */
  float mu0;         /* step size cap (the paper's mu)                                            */
  double lamA;       /* upper bound on lambda_max(A^H A); <= 0 keeps mu = mu0                      */
  float sigma2;      /* sigma^2 of eq. (8); <= 0 selects the median rule                           */
  int n_max;         /* maximum number of iterations                                              */
  double tol;        /* stopping tolerance; < 0 runs exactly n_max iterations                     */
  int serial;        /* 0: independent parts of an iteration overlap on two streams the recon owns
                        (the cost terms of X; the graph rebuild and the SVT coefficients beside the
                        gradient). Bit 0 keeps the cost terms, bit 1 the rest on the caller's
                        stream (per-kernel timings then carry no overlap). Results are identical.  */
} mrf_recon_params;

#define MRF_MAX_ITERS 512
typedef struct mrf_recon_stats {
  int iters;         /* iterations run                                                            */
  int stop_reason;   /* 0: n_max reached, 1: tolerance met                                        */
  int n_graph;       /* graphs built                                                              */
  double cost[MRF_MAX_ITERS + 1];   /* cost(0 .. iters)                                         */
  double data[MRF_MAX_ITERS + 1];   /* 1/2 ||A X - b||^2                                        */
  double tr[MRF_MAX_ITERS + 1];     /* Tr(Q(X) L Q(X)^H)                                        */
  double nuc[MRF_MAX_ITERS + 1];    /* sum_i ||Q_i X||_*                                        */
  double mu[MRF_MAX_ITERS + 1];     /* per graph: step size, lambda1, sigma^2, max(L)          */
  double lam1[MRF_MAX_ITERS + 1];
  double sigma2[MRF_MAX_ITERS + 1];
  double lmax[MRF_MAX_ITERS + 1];
  double iter_ms[MRF_MAX_ITERS + 1]; /* host wall time of iteration n (1 .. iters): from its first
                                        enqueued kernel to its cost on the host; [0]: initialisation */
} mrf_recon_stats;

typedef struct mrf_recon_s* mrf_recon_t;

/* Allocates the solver state (device memory owned by the handle, about 2 images of L x n x n
 * plus the NUFFT and LLR work buffers) for a plan and a dictionary created with a basis V. */
mrf_status mrf_recon_create(const mrf_recon_params* prm, mrf_nufft_plan_t plan, mrf_dict_t dict, mrf_recon_t* out);
mrf_status mrf_recon_destroy(mrf_recon_t r);
/* Initialisation of Algorithm 1 with measurements b [L][Ns] (kept by pointer until the last
 * call that uses it) and an optional X0 [L][n][n] (NULL: X0 = A^H b). Synchronises. */
mrf_status mrf_recon_init(mrf_recon_t r, const mrf_c64* b, const mrf_c64* X0, hipStream_t stream);
/* Multi-coil data (eq. (1)): from the next mrf_recon_init on, the data term is
 * 0.5 ||F_u C X - b||^2 with C the coil sensitivities smaps [ncoils][n][n] (device complex64,
 * copied here; the caller's buffer may be freed afterwards), b then holds ncoils series
 * [ncoils][L][Ns], X0 = A^H b is the coil-combined adjoint and lamA must bound
 * lambda_max((F_u C)^H F_u C) (mrf_nufft_opnorm_mc). smaps NULL returns to a single coil. Clears
 * the initialised state (call mrf_recon_init again); allocates the residual for all coils and
 * synchronises. A checkpoint records the coil count and loads only into a recon with the same
 * count. MRF_INVALID_ARG for a null handle or ncoils < 1 with maps, MRF_OOM. */
mrf_status mrf_recon_set_coils(mrf_recon_t r, const mrf_c64* smaps, int ncoils, hipStream_t stream);
/* Toeplitz normal operator in Algorithm 1 (the gradient of eq. (15)): from the next
 * mrf_recon_init on, the data term's gradient is A^H A X - A^H b with A^H A X from
 * mrf_toeplitz_normal (t, made from the plan's own desc and trajectory; handle kept by pointer),
 * and its value is 0.5 (<X, A^H A X> - 2 Re <X, A^H b> + ||b||^2): no forward transform runs in
 * the loop and A^H only once, at initialisation. Each iteration applies A^H A once, to X^{n+1}
 * for its cost, and the next gradient reuses it. The iterates equal the gridded pair's to the
 * KB error; the data term's value loses about 1e-7 of ||A X||^2 to the cancellation of its three
 * parts (accumulated in FP64 from FP32 inputs). t NULL returns to the gridded pair. Single coil
 * only: MRF_NOT_SUPPORTED with coil maps set (and set_coils refuses while t is set);
 * MRF_SHAPE if t's n or frame count differ or its workspace exceeds the plan's. Clears the
 * initialised state; allocates two image series; synchronises. A checkpoint restores into a
 * recon in the same mode (A^H b and A^H A X are recomputed from b and X). */
mrf_status mrf_recon_set_toeplitz(mrf_recon_t r, mrf_toeplitz_t t, hipStream_t stream);
/* Runs up to n more iterations (stops early on the tolerance or at n_max). Synchronises once
 * per iteration to read the cost. *stopped (may be NULL) is set when no iteration is left. */
mrf_status mrf_recon_iterate(mrf_recon_t r, int n, int* stopped, hipStream_t stream);
/* Sets mrf_recon_params.serial for the iterations that follow (an iteration leaves no work
 * on the recon's own streams once its cost has been read, so the schedule may change between
 * calls). Host only; MRF_INVALID_ARG for a null handle. */
mrf_status mrf_recon_set_serial(mrf_recon_t r, int serial);
/* C5: advances nslices independent reconstructions (each created and initialised on its own,
 * with its own plan, dictionary and graph; slices may differ in n, L and Ns) by up to n
 * iterations each. Per round, every active slice's iteration is enqueued on its own stream
 * (streams[i], default priority), then each is waited for and its stopping rule applied, so the
 * slices' kernels overlap on the device. n_active (host, optional): slices still running. */
mrf_status mrf_recon_batched(int nslices, const mrf_recon_t* recons, const hipStream_t* streams, int n, int* n_active);
/* Final match Phi_D(X): any of X_out [L][n][n], maps [3][n][n] (T1, T2, PD), idx [n*n],
 * rho [n*n] may be NULL. Asynchronous. */
mrf_status mrf_recon_finish(mrf_recon_t r, mrf_c64* X_out, float* maps, int32_t* idx, float* rho, hipStream_t stream);
/* Parity diagnostic: graph number k (k = 0: the graph built at mrf_recon_init from M^0;
 * k = n: the graph built from M^n before iteration n + 1) is not built from the match but taken
 * as given: the Laplacian L in CSR (host arrays: rowptr [Np + 1] from 0 to nnz, col [nnz]
 * ascending within each row with the diagonal present, val [nnz] = entries of L), with its sigma^2
 * and max(L) (which set lambda1 and mu). The match M^k is still computed. Lets a run follow an
 * external reference's graphs so that floating-point drift is told apart from discrete changes of
 * the graph (arg-max and K-NN near-ties). Copies the arrays to device memory owned by the recon
 * (synchronous); a later call for the same k replaces the earlier one. MRF_SHAPE if nnz exceeds
 * the graph's capacity (Np (2 K + 1)). */
mrf_status mrf_recon_inject_graph(mrf_recon_t r, int k, int nnz, const int* rowptr, const int* col, const float* val,
                                  double sigma2, double lmax);
/* The final match Phi_D(X^) of Algorithm 1 (mrf_recon_finish and mrf_recon): MRF_MATCH_SUBSPACE
 * (default; the subspace match used inside the loop), MRF_MATCH_FP32 / _BF16_RERANK4 /
 * _FP8_RERANK4 (the full-length match of mrf_dict_match on X^'s voxel time courses), or
 * MRF_MATCH_LEARNED (mrf_mlp_match on X^ V with gate threshold theta; mlp must have its grid set
 * and be trained for the dictionary's basis). maps [3][n][n] then hold (T1, T2) of the chosen
 * match and PD = rho. Allocates the work buffers the mode needs (recon-owned; replaced by a later
 * call, freed by mrf_recon_destroy) and synchronises. With MRF_MATCH_LEARNED, mrf_recon_finish
 * synchronises once (the fallback count). */
mrf_status mrf_recon_set_final_match(mrf_recon_t r, mrf_match_mode mode, mrf_mlp_t mlp, float theta);
/* Checkpoint of a run between iterations (after mrf_recon_init or mrf_recon_iterate): X^n, the
 * residual A X^n - b, the eigen-analysis of Q(X^n) that the next SVT uses, the device scalars,
 * the statistics and the stopping state. mrf_recon_checkpoint_bytes gives the size; save writes it
 * to buf (host or device memory, at least that many bytes) and synchronises `stream`. load
 * restores it into a recon created with the same parameters, plan and dictionary (checked against
 * the sizes recorded in buf; MRF_SHAPE otherwise), with the measurements b of the run; the
 * iterations that follow give bit-for-bit the same results as the uninterrupted run. */
mrf_status mrf_recon_checkpoint_bytes(mrf_recon_t r, size_t* bytes);
mrf_status mrf_recon_checkpoint_save(mrf_recon_t r, void* buf, size_t bytes, hipStream_t stream);
mrf_status mrf_recon_checkpoint_load(mrf_recon_t r, const mrf_c64* b, const void* buf, size_t bytes, hipStream_t stream);
/* Copies the statistics of the run so far (host struct). */
mrf_status mrf_recon_get_stats(mrf_recon_t r, mrf_recon_stats* out);
/* The whole of Algorithm 1: init + iterate(n_max) + finish; stats may be NULL. */
mrf_status mrf_recon(mrf_recon_t r, const mrf_c64* b, const mrf_c64* X0, mrf_c64* X_out, float* maps, int32_t* idx,
                     float* rho, mrf_recon_stats* stats, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MRF_H */
