// FISP signal model by the extended phase graph (eqs. (2)-(3)): the step that makes the dictionary
// atoms d_m = B(eta_m; theta) (PD = 1) and off-grid training signals, on the device.
//
// Model: configuration states F+_k, F-_k, Z_k, k < K. An ideal inversion and one TR of recovery;
// then per frame l an RF rotation about x by a_l = FA_l B1 (every k mixed by the same 3 x 3
// matrix), the signal F+_0 exp(-TE/T2), relaxation over TR_l (recovery into Z_0), and one
// dephasing shift (F+ up one order, F- down one order, F+_0 = conj(F-_0)); orders >= K drop out.
//
// One thread per parameter set with its 3K complex states in registers (K a template constant,
// so every state index is static and the shift is register renaming). The train (FA, TR) is the
// same for every thread: uniform loads. Signals are staged in LDS for 16 frames and written
// atom-major, 128 contiguous bytes per atom and stage.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"
#include "philox.hpp"

namespace mrf {

constexpr int kEpgBlock = 256;
constexpr int kEpgStage = 16;   // frames per staged write

template <int K>
__global__ __launch_bounds__(kEpgBlock) void k_epg(int M, int L, const float* __restrict__ t1,
                                                   const float* __restrict__ t2, const float* __restrict__ b1,
                                                   const float* __restrict__ fa_deg, const float* __restrict__ tr_ms,
                                                   float te_ms, cf* __restrict__ out) {
  __shared__ cf stage[kEpgStage][kEpgBlock + 1];
  const int tid = threadIdx.x;
  const long m0 = (long)blockIdx.x * kEpgBlock;
  const bool valid = m0 + tid < M;
  const float T1 = valid ? t1[m0 + tid] : 1000.f, T2 = valid ? t2[m0 + tid] : 100.f;
  const float scale = (valid && b1) ? b1[m0 + tid] : 1.f;
  const float r1 = 1.0f / T1, r2 = 1.0f / T2;
  const float ete = expf(-te_ms * r2);
  const float deg = scale * 0.017453292519943295f;   // pi / 180
  float fpr[K], fpi[K], fmr[K], fmi[K], zr[K], zi[K];
#pragma unroll
  for (int k = 0; k < K; ++k) fpr[k] = fpi[k] = fmr[k] = fmi[k] = zr[k] = zi[k] = 0.f;
  {
    const float e1 = expf(-tr_ms[0] * r1);
    zr[0] = 1.0f - 2.0f * e1;   // inversion, one TR of recovery
  }
  for (int l0 = 0; l0 < L; l0 += kEpgStage) {
    const int nf = min(kEpgStage, L - l0);
    for (int j = 0; j < nf; ++j) {
      const int l = l0 + j;
      float sa, ca;
      sincosf(fa_deg[l] * deg, &sa, &ca);
      const float c2 = 0.5f * (1.0f + ca), s2 = 0.5f * (1.0f - ca), hs = 0.5f * sa;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float pr = fpr[k], pi = fpi[k], qr = fmr[k], qi = fmi[k], wr = zr[k], wi = zi[k];
        // F+' = c2 F+ + s2 F- - i sa Z ; F-' = s2 F+ + c2 F- + i sa Z
        fpr[k] = c2 * pr + s2 * qr + sa * wi;
        fpi[k] = c2 * pi + s2 * qi - sa * wr;
        fmr[k] = s2 * pr + c2 * qr - sa * wi;
        fmi[k] = s2 * pi + c2 * qi + sa * wr;
        // Z' = -(i/2) sa F+ + (i/2) sa F- + ca Z
        zr[k] = hs * (pi - qi) + ca * wr;
        zi[k] = hs * (qr - pr) + ca * wi;
      }
      stage[j][tid] = cf{fpr[0] * ete, fpi[0] * ete};
      const float tr = tr_ms[l];
      const float E1 = expf(-tr * r1), E2 = expf(-tr * r2);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        fpr[k] *= E2; fpi[k] *= E2; fmr[k] *= E2; fmi[k] *= E2;
        zr[k] *= E1; zi[k] *= E1;
      }
      zr[0] += 1.0f - E1;
#pragma unroll
      for (int k = K - 1; k >= 1; --k) {
        fpr[k] = fpr[k - 1];
        fpi[k] = fpi[k - 1];
      }
#pragma unroll
      for (int k = 0; k < K - 1; ++k) {
        fmr[k] = fmr[k + 1];
        fmi[k] = fmi[k + 1];
      }
      fmr[K - 1] = 0.f;
      fmi[K - 1] = 0.f;
      fpr[0] = fmr[0];
      fpi[0] = -fmi[0];
    }
    __syncthreads();
    for (int idx = tid; idx < kEpgBlock * kEpgStage; idx += kEpgBlock) {
      const int a = idx / kEpgStage, j = idx % kEpgStage;
      if (j < nf && m0 + a < M) out[(m0 + a) * L + l0 + j] = stage[j][a];
    }
    __syncthreads();
  }
}

// Off-grid parameters: for set i, Philox4x32-10 with counter (i, 0x45504731, 0, 0) and key
// (seed low, seed high) gives u1, u2, u3 in (0, 1); T1 = exp(log t1_lo + u1 (log t1_hi - log t1_lo)),
// T2 = exp(log t2_lo + u2 (log min(t2_hi, T1) - log t2_lo)) (so T2 <= T1, the rule of the paper's
// dictionary), B1 = b1_lo + u3 (b1_hi - b1_lo). params [n][3] = (T1, T2, B1).
__global__ void k_epg_params(int n, unsigned k0, unsigned k1, float lt1a, float lt1b, float t2a, float t2b,
                             float b1a, float b1b, float* __restrict__ params) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const u4 u = philox(u4{(unsigned)i, 0x45504731u, 0u, 0u}, k0, k1);
  const float T1 = expf(lt1a + u01(u.x) * (lt1b - lt1a));
  const float l2a = logf(t2a), l2b = logf(fminf(t2b, T1));
  const float T2 = expf(l2a + u01(u.y) * (l2b - l2a));
  params[3 * i + 0] = T1;
  params[3 * i + 1] = T2;
  params[3 * i + 2] = b1a + u01(u.z) * (b1b - b1a);
}

// T1, T2, B1 columns of params [n][3] for the simulator
__global__ void k_split_params(int n, const float* __restrict__ params, float* __restrict__ cols) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cols[i] = params[3 * i];
  cols[n + i] = params[3 * i + 1];
  cols[2 * n + i] = params[3 * i + 2];
}

namespace {
template <int K>
void launch_epg(int M, int L, const float* t1, const float* t2, const float* b1, const float* fa, const float* tr,
                float te, cf* out, hipStream_t s) {
  MRF_LAUNCH("epg_fisp", s, k_epg<K><<<ceil_div(M, kEpgBlock), kEpgBlock, 0, s>>>(M, L, t1, t2, b1, fa, tr, te, out));
}
}  // namespace

}  // namespace mrf

using namespace mrf;

extern "C" mrf_status mrf_epg_fisp(int n_atoms, int n_frames, int n_states, const float* t1, const float* t2,
                                   const float* b1, const float* fa_deg, const float* tr_ms, float te_ms,
                                   mrf_c64* out, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(t1 && t2 && fa_deg && tr_ms && out, MRF_INVALID_ARG, "epg_fisp: null argument");
  MRF_REQUIRE(n_atoms >= 1 && n_frames >= 1, MRF_INVALID_ARG, "epg_fisp: n_atoms, n_frames must be >= 1");
  MRF_REQUIRE(te_ms >= 0.f, MRF_INVALID_ARG, "epg_fisp: te_ms must be >= 0");
  cf* o = (cf*)out;
  switch (n_states) {
    case 8: launch_epg<8>(n_atoms, n_frames, t1, t2, b1, fa_deg, tr_ms, te_ms, o, s); break;
    case 16: launch_epg<16>(n_atoms, n_frames, t1, t2, b1, fa_deg, tr_ms, te_ms, o, s); break;
    case 24: launch_epg<24>(n_atoms, n_frames, t1, t2, b1, fa_deg, tr_ms, te_ms, o, s); break;
    case 32: launch_epg<32>(n_atoms, n_frames, t1, t2, b1, fa_deg, tr_ms, te_ms, o, s); break;
    default: return fail(MRF_SHAPE, "epg_fisp: n_states must be 8, 16, 24 or 32");
  }
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

extern "C" mrf_status mrf_epg_random_params(int n, uint64_t seed, float t1_lo, float t1_hi, float t2_lo, float t2_hi,
                                            float b1_lo, float b1_hi, float* params, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(params && n >= 1, MRF_INVALID_ARG, "epg_random_params: null params or n < 1");
  MRF_REQUIRE(t1_lo > 0.f && t1_hi >= t1_lo && t2_lo > 0.f && t2_hi >= t2_lo && t2_lo <= t1_lo && b1_hi >= b1_lo,
              MRF_INVALID_ARG, "epg_random_params: need 0 < t2_lo <= t1_lo <= t1_hi, t2_lo <= t2_hi, b1_lo <= b1_hi");
  MRF_LAUNCH("epg_params", s,
             k_epg_params<<<ceil_div(n, 256), 256, 0, s>>>(n, (unsigned)seed, (unsigned)(seed >> 32), logf(t1_lo),
                                                           logf(t1_hi), t2_lo, t2_hi, b1_lo, b1_hi, params));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

extern "C" mrf_status mrf_epg_params_to_columns(int n, const float* params, float* cols, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(params && cols && n >= 1, MRF_INVALID_ARG, "epg_params_to_columns: null argument or n < 1");
  MRF_LAUNCH("epg_params", s, k_split_params<<<ceil_div(n, 256), 256, 0, s>>>(n, params, cols));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}
