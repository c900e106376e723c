// Algorithm 1 (MS-LLR reconstruction, Sec. III-C/D) on the device.
//
//   X^0 = A^H b, M^0 = Phi_D(X^0), L^0 from M^0, lambda1 = lambda1^0 max(L^0)
//   each iteration:
//     Z^n     = P_S(X^n - mu [A^H(A X^n - b) + lambda1 Q*(Q(X^n) L^n)])        eq. (15)
//     P^{n+1} = SVT_{1/beta}(Q_q(X^n)) on every patch                          eq. (22)
//     X^{n+1} = (Z^n + mu lam2 beta Q*(P^{n+1})) / (1 + mu lam2 beta c)        eq. (23)
//     cost    = 1/2 ||A X^{n+1} - b||^2 + lambda1 Tr(Q L^n Q^H) + lam2 sum ||Q_q X^{n+1}||_*
//     stop if cost(n)/cost(n+1) - 1 < tol; else M^{n+1} = Phi_D(X^{n+1}), L^{n+1}, lambda1, mu
// Exactly one forward and one adjoint NUFFT per iteration: A X^{n+1} of the cost is the next
// gradient's residual. The Laplacian term of the gradient is applied in the subspace:
// P_S(Q*(Q(X) L)) = S_L(X V) V^H, because S_L acts on pixels and V on frames, so S_L runs on
// r coefficient images instead of L frames. The eigen-analysis of Q(X^{n+1}) serves both the
// cost's nuclear norm and the next SVT. The only device-to-host traffic is the cost terms,
// once per iteration (the stopping rule).
// Readings: the SVT acts on Q(X^n) (eq. (22)); eq. (23) divides per pixel by 1 + mu lam2 beta c(v)
// (the exact minimiser of eq. (21) for overlapping patches); mu = min(mu0, 1/(lamA + 2 c_max
// lambda1 max(L))) with lamA a bound on lambda_max(A^H A) (mu = mu0 when lamA <= 0).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "dict.hpp"
#include "patch.hpp"

namespace mrf {
// nufft.hip
mrf_status nufft_residual(const mrf_nufft_plan_s* p, const cf* img, const cf* b, cf* r, void* ws, double* part,
                          double* rn2, hipStream_t s, const cf* smaps, int ncoils);
mrf_status nufft_adj_coils(const mrf_nufft_plan_s* p, const cf* ksp, cf* img, void* ws, hipStream_t s,
                           const cf* smaps, int ncoils);
mrf_status sum_partials(const double* part, long n, double* out, hipStream_t s);
// toeplitz.hip
mrf_status toeplitz_apply(const mrf_toeplitz_s* T, const cf* X, cf* Y, void* ws, hipStream_t s);
size_t toeplitz_ws_bytes(const mrf_toeplitz_s* T);
int toeplitz_n(const mrf_toeplitz_s* T);
int toeplitz_frames(const mrf_toeplitz_s* T);
long nufft_resid_blocks(const mrf_nufft_plan_s* p);
int nufft_n(const mrf_nufft_plan_s* p);
int nufft_frames(const mrf_nufft_plan_s* p);
int nufft_nsamp(const mrf_nufft_plan_s* p);
size_t nufft_ws_bytes(const mrf_nufft_plan_s* p);
// graph.hip
mrf_status graph_build(mrf_graph_s* G, const float* maps, int K, float sigma2, hipStream_t s);
mrf_status lap_quad(mrf_graph_s* G, const cf* X, int L, double* out, hipStream_t s);
mrf_status lap_apply_sub(const mrf_graph_s* G, const cf* A, cf* Y, int r, hipStream_t s);
const double* graph_scalars(const mrf_graph_s* G);
size_t graph_capacity(const mrf_graph_s* G);
mrf_status graph_set_csr(mrf_graph_s* G, const int* rowptr, const int* col, const float* val, int nnz,
                         const double* scal, hipStream_t s);
// subspace.hip
size_t reduce_ws_bytes(int L, int Nv, int r);
mrf_status subspace_reduce(const cf* X, const cf* Gd, const double* mu_dev, const cf* V, int L, int Nv, int r,
                           cf* alpha, cf* part, hipStream_t s);
mrf_status subspace_expand(const cf* beta, const cf* V, int L, int Nv, int r, cf* Z, hipStream_t s);
mrf_status axpy_scal(const cf* aU, const cf* Y, const double* s0, const double* s1, double scale, long n, cf* out,
                     hipStream_t s);
mrf_status grad_coef(const cf* aX, const cf* aG, const cf* Y, const double* mu, const double* lam1, long n, cf* out,
                     hipStream_t s);
mrf_status match_subspace(const mrf_dict_s* D, const cf* alpha, int Nv, int* idx, float* rho, float* score,
                          float* params, hipStream_t s);
mrf_status maps_from_match(const mrf_dict_s* D, const int* idx, const float* rho, int Nv, float* maps, hipStream_t s);
const cf* dict_basis(const mrf_dict_s* D);
int dict_rank(const mrf_dict_s* D);
int dict_frames(const mrf_dict_s* D);
// llr.hip
size_t llr_ws_bytes(const PatchGeom& g, int rcap);
mrf_status llr_analyse(const cf* X, const PatchGeom& g, int L, double tau, int rcap, void* ws, cf* U, float* f,
                       double* nuc_out, double* lam_out, hipStream_t s);
mrf_status llr_coef(const cf* X, const PatchGeom& g, int L, int rcap, const cf* U, const float* f, cf* C, hipStream_t s);
bool llr_xupdate_beta_ok(const PatchGeom& g, int rcap, int r);
mrf_status llr_xupdate_beta(const cf* beta, const cf* V, int r, const cf* U, const cf* C, const PatchGeom& g, int L,
                            int rcap, const double* kap_dev, double kap_scale, cf* Xout, hipStream_t s);
mrf_status llr_xupdate(const cf* Z, const cf* U, const cf* C, const PatchGeom& g, int L, int rcap,
                       const double* kap_dev, double kap_scale, cf* Xout, hipStream_t s);

// device scalars
enum { SC_LAM1 = 0, SC_MU, SC_KAP, SC_LMAX, SC_RN2, SC_QUAD, SC_NUC, SC_COST, SC_SIGMA2, SC_N = 16 };

__global__ void k_scalars(const double* __restrict__ gs, double* __restrict__ sc, double lam1_0, double lamA,
                          double cmax, double mu0, double lam2, double beta) {
  const double lmax = gs[1];
  const double lam1 = lam1_0 * lmax;
  double mu = mu0;
  if (lamA > 0.0) mu = fmin(mu0, 1.0 / (lamA + 2.0 * cmax * lam1 * lmax));
  sc[SC_LAM1] = lam1;
  sc[SC_MU] = mu;
  sc[SC_KAP] = mu * lam2 * beta;
  sc[SC_LMAX] = lmax;
  sc[SC_SIGMA2] = gs[0];
}

__global__ void k_cost(double* __restrict__ sc, double lam2) {
  sc[SC_COST] = 0.5 * sc[SC_RN2] + sc[SC_LAM1] * sc[SC_QUAD] + lam2 * sc[SC_NUC];
}

// maps [3][Nv] = (T1, T2) from per-voxel parameter rows (stride np) and PD = rho
__global__ void k_maps_params(const float* __restrict__ prm, int np, const float* __restrict__ rho, int Nv,
                              float* __restrict__ maps) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= Nv) return;
  maps[v] = prm[(size_t)v * np];
  maps[Nv + v] = prm[(size_t)v * np + 1];
  maps[2 * Nv + v] = rho[v];
}

// Toeplitz data term: block partials of Re<x, A^H A x> - 2 Re<x, A^H b> (each block a fixed
// grid-stride share, summed in a fixed order), so that adding ||b||^2 gives ||A x - b||^2.
constexpr int kToepDataBlocks = 1024;
__global__ __launch_bounds__(256) void k_toep_data(const cf* __restrict__ X, const cf* __restrict__ TX,
                                                   const cf* __restrict__ AHb, long n, double* __restrict__ part) {
  __shared__ double red[4];
  double q = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const cf x = X[i], t = TX[i], a = AHb[i];
    q += (double)x.x * t.x + (double)x.y * t.y - 2.0 * ((double)x.x * a.x + (double)x.y * a.y);
  }
  for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// sum of |b|^2 in the same blocked order
__global__ __launch_bounds__(256) void k_norm2(const cf* __restrict__ b, long n, double* __restrict__ part) {
  __shared__ double red[4];
  double q = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    q += (double)b[i].x * b[i].x + (double)b[i].y * b[i].y;
  for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_add_scalar(double* __restrict__ a, const double* __restrict__ b) { a[0] += b[0]; }

__global__ void k_sub_c(cf* __restrict__ a, const cf* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = cf{a[i].x - b[i].x, a[i].y - b[i].y};
}

__global__ void k_copy_c(const cf* __restrict__ a, cf* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = a[i];
}

}  // namespace mrf

using namespace mrf;

struct mrf_recon_s {
  mrf_recon_params prm;
  mrf_nufft_plan_s* plan;
  mrf_dict_s* dict;
  mrf_graph_s* graph;
  PatchGeom g;
  int N, L, Ns, Nv, r;
  double cmax;
  const cf* b;
  cf *X, *ZG, *res, *aX, *aU, *Ya, *beta, *U, *C;
  float *f, *maps, *rho;
  int* idx;
  void *nws, *rws, *rws2, *lws;   // rws2: the graph rebuild's reduction, which overlaps the gradient's
  double *sc, *rpart;
  // Independent parts of an iteration run on two streams of the recon beside the caller's stream
  // (default priority), forked from and joined back into it by events.
  hipStream_t aux[2];
  hipEvent_t ev_fork, ev_aux[2];
  bool initialised;
  bool pending_graph;   // a rebuilt graph whose scalars are not yet recorded
  double* hsc;          // pinned host copy of the device scalars
  double c_prev;
  mrf_recon_stats st;
  std::vector<void*> allocs;
  // graphs supplied by mrf_recon_inject_graph, by graph number (device copies owned here)
  struct Injected {
    int k, nnz;
    int *rowptr, *col;
    float* val;
    double* scal;
  };
  std::vector<Injected> inj;
  // the final match (mrf_recon_set_final_match)
  int fin_mode = MRF_MATCH_SUBSPACE;
  mrf_mlp_t fin_mlp = nullptr;
  float fin_theta = 0.f;
  void* fin_ws = nullptr;
  size_t fin_ws_bytes = 0;
  float* fin_prm = nullptr;     // [Nv][nparam] (full-length modes) or [Nv][2] (learned)
  std::chrono::steady_clock::time_point t_step;   // enqueue time of the iteration in flight
  // coil sensitivities (mrf_recon_set_coils): a device copy, and the residual and its block
  // partials sized for all coils; res1 / rpart1 are the single-coil buffers of mrf_recon_create
  cf* smaps = nullptr;
  int ncoils = 0;
  cf* res1 = nullptr;
  double* rpart1 = nullptr;
  std::vector<void*> coil_bufs;
  // Toeplitz normal operator (mrf_recon_set_toeplitz): T(X), A^H b, (A^H b) V, ||b||^2 and the
  // data term's block partials; its workspace is the NUFFT workspace, idle in this mode
  mrf_toeplitz_s* toep = nullptr;
  cf *TX = nullptr, *AHb = nullptr, *AHbV = nullptr;
  double *tpart = nullptr, *bn2 = nullptr;
  std::vector<void*> toep_bufs;
};

namespace {

// Stream for aux part k of a phase (bit = the phase's bit of prm.serial): s when serial.
hipStream_t aux_stream(const mrf_recon_s* R, int k, int bit, hipStream_t s) {
  return (R->prm.serial & bit) ? s : R->aux[k];
}
// aux streams start after the work enqueued so far on s
mrf_status fork(mrf_recon_s* R, int bit, hipStream_t s) {
  if (R->prm.serial & bit) return MRF_OK;
  MRF_CHECK_HIP(hipEventRecord(R->ev_fork, s));
  for (int k = 0; k < 2; ++k) MRF_CHECK_HIP(hipStreamWaitEvent(R->aux[k], R->ev_fork, 0));
  return MRF_OK;
}
// work enqueued later on s waits for what aux stream k holds so far
mrf_status join(mrf_recon_s* R, int k, int bit, hipStream_t s) {
  if (R->prm.serial & bit) return MRF_OK;
  MRF_CHECK_HIP(hipEventRecord(R->ev_aux[k], R->aux[k]));
  MRF_CHECK_HIP(hipStreamWaitEvent(s, R->ev_aux[k], 0));
  return MRF_OK;
}

const mrf_recon_s::Injected* injected(const mrf_recon_s* R, int k) {
  for (const auto& g : R->inj)
    if (g.k == k) return &g;
  return nullptr;
}

// M = Phi_D(X) and the graph built from it (graph number R->st.n_graph: 0 at the initialisation,
// n before iteration n + 1), or the graph supplied for that number; then lambda1 and mu.
mrf_status rebuild(mrf_recon_s* R, hipStream_t s) {
  mrf_status e;
  if ((e = subspace_reduce(R->X, nullptr, nullptr, dict_basis(R->dict), R->L, R->Nv, R->r, R->aX, (cf*)R->rws2, s)))
    return e;
  if ((e = match_subspace(R->dict, R->aX, R->Nv, R->idx, R->rho, nullptr, nullptr, s))) return e;
  if ((e = maps_from_match(R->dict, R->idx, R->rho, R->Nv, R->maps, s))) return e;
  if (const auto* ig = injected(R, R->st.n_graph))
    e = graph_set_csr(R->graph, ig->rowptr, ig->col, ig->val, ig->nnz, ig->scal, s);
  else
    e = graph_build(R->graph, R->maps, R->prm.K, R->prm.sigma2, s);
  if (e) return e;
  MRF_LAUNCH("recon_scalars", s,
             k_scalars<<<1, 1, 0, s>>>(graph_scalars(R->graph), R->sc, R->prm.lam1_0, R->prm.lamA, R->cmax, R->prm.mu0,
                                       R->prm.lam2, R->prm.beta));
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

// cost terms of the current X (with the current graph), copied to the pinned host scalars. The three
// terms only read X: the residual runs on s, the eigen-analysis (which also gives the next SVT's U
// and f) on aux[0] and the Laplacian trace on aux[1], each into buffers of its own.
mrf_status evaluate_enqueue(mrf_recon_s* R, hipStream_t s) {
  mrf_status e;
  if ((e = fork(R, 1, s))) return e;
  if ((e = llr_analyse(R->X, R->g, R->L, 1.0 / R->prm.beta, R->prm.rank_cap, R->lws, R->U, R->f, R->sc + SC_NUC,
                       nullptr, aux_stream(R, 0, 1, s))))
    return e;
  if ((e = lap_quad(R->graph, R->X, R->L, R->sc + SC_QUAD, aux_stream(R, 1, 1, s)))) return e;
  if (R->toep) {
    // ||A X - b||^2 = <X, A^H A X> - 2 Re <X, A^H b> + ||b||^2; A^H A X is kept for the next gradient
    if ((e = toeplitz_apply(R->toep, R->X, R->TX, R->nws, s))) return e;
    MRF_LAUNCH("recon_toep_data", s, k_toep_data<<<kToepDataBlocks, 256, 0, s>>>(R->X, R->TX, R->AHb,
                                                                                (long)R->L * R->Nv, R->tpart));
    if ((e = sum_partials(R->tpart, kToepDataBlocks, R->sc + SC_RN2, s))) return e;
    MRF_LAUNCH("recon_toep_data", s, k_add_scalar<<<1, 1, 0, s>>>(R->sc + SC_RN2, R->bn2));
  } else if ((e = nufft_residual(R->plan, R->X, R->b, R->res, R->nws, R->rpart, R->sc + SC_RN2, s, R->smaps,
                                 R->ncoils))) {
    return e;
  }
  if ((e = join(R, 0, 1, s)) || (e = join(R, 1, 1, s))) return e;
  MRF_LAUNCH("recon_cost", s, k_cost<<<1, 1, 0, s>>>(R->sc, R->prm.lam2));
  MRF_CHECK_LAUNCH();
  MRF_CHECK_HIP(hipMemcpyAsync(R->hsc, R->sc, SC_N * sizeof(double), hipMemcpyDeviceToHost, s));
  return MRF_OK;
}

// the same, waiting for the result
mrf_status evaluate(mrf_recon_s* R, hipStream_t s, double* h) {
  mrf_status e = evaluate_enqueue(R, s);
  if (e) return e;
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  std::copy(R->hsc, R->hsc + SC_N, h);
  if (!std::isfinite(h[SC_COST])) return fail(MRF_NONFINITE, "recon: cost is not finite");
  return MRF_OK;
}

void record(mrf_recon_s* R, const double* h, bool graph_row) {
  const int n = R->st.iters;
  if (n <= MRF_MAX_ITERS) {
    R->st.cost[n] = h[SC_COST];
    R->st.data[n] = 0.5 * h[SC_RN2];
    R->st.tr[n] = h[SC_QUAD];
    R->st.nuc[n] = h[SC_NUC];
  }
  (void)graph_row;
}

void record_graph(mrf_recon_s* R, const double* h) {
  const int n = R->st.n_graph;
  if (n <= MRF_MAX_ITERS) {
    R->st.mu[n] = h[SC_MU];
    R->st.lam1[n] = h[SC_LAM1];
    R->st.sigma2[n] = h[SC_SIGMA2];
    R->st.lmax[n] = h[SC_LMAX];
    R->st.n_graph = n + 1;
  }
}

// Toeplitz mode: A^H b (reusing X^0 when it is A^H b), (A^H b) V and ||b||^2 for the data term
mrf_status toep_prepare(mrf_recon_s* R, bool x_is_ahb, hipStream_t s) {
  mrf_status e;
  if (x_is_ahb) {
    MRF_LAUNCH("recon_copy", s, k_copy_c<<<1024, 256, 0, s>>>(R->X, R->AHb, (size_t)R->L * R->Nv));
  } else if ((e = nufft_adj_coils(R->plan, R->b, R->AHb, R->nws, s, nullptr, 0))) {
    return e;
  }
  if ((e = subspace_reduce(R->AHb, nullptr, nullptr, dict_basis(R->dict), R->L, R->Nv, R->r, R->AHbV, (cf*)R->rws,
                           s)))
    return e;
  MRF_LAUNCH("recon_toep_data", s, k_norm2<<<kToepDataBlocks, 256, 0, s>>>(R->b, (long)R->L * R->Ns, R->tpart));
  if ((e = sum_partials(R->tpart, kToepDataBlocks, R->bn2, s))) return e;
  MRF_CHECK_LAUNCH();
  return MRF_OK;
}

}  // namespace

extern "C" mrf_status mrf_recon_create(const mrf_recon_params* prm, mrf_nufft_plan_t plan, mrf_dict_t dict,
                                       mrf_recon_t* out) {
  clear_error();
  MRF_REQUIRE(prm && plan && dict && out, MRF_INVALID_ARG, "recon_create: null argument");
  *out = nullptr;
  const int N = nufft_n(plan), L = nufft_frames(plan), Ns = nufft_nsamp(plan);
  MRF_REQUIRE(dict_rank(dict) > 0, MRF_INVALID_ARG, "recon_create: the dictionary needs a subspace basis V");
  MRF_REQUIRE(dict_frames(dict) == L, MRF_SHAPE, "recon_create: dictionary length differs from the plan's frames");
  MRF_REQUIRE(N % 16 == 0, MRF_SHAPE, "recon_create: n must be a multiple of 16");
  MRF_REQUIRE(prm->beta > 0.f && prm->mu0 > 0.f && prm->lam2 >= 0.f && prm->lam1_0 >= 0.f, MRF_INVALID_ARG,
              "recon_create: need beta > 0, mu0 > 0, lam1_0 >= 0, lam2 >= 0");
  MRF_REQUIRE(prm->n_max >= 0, MRF_INVALID_ARG, "recon_create: n_max must be >= 0");
  auto* R = new mrf_recon_s{};
  R->prm = *prm;
  R->plan = plan;
  R->dict = dict;
  R->N = N; R->L = L; R->Ns = Ns; R->Nv = N * N; R->r = dict_rank(dict);
  mrf_status st = mrf_graph_create(N, prm->p, prm->s, std::max(1, prm->K), L, &R->graph);
  if (st != MRF_OK) {
    delete R;
    return st;
  }
  make_geom(N, prm->p, prm->s, &R->g);
  const int pp = prm->p * prm->p;
  if (!((pp == 16 || pp == 64 || pp < 16) && prm->rank_cap >= 1 && prm->rank_cap <= 16 && prm->K >= 1 &&
        prm->K <= R->g.Np - 1)) {
    mrf_graph_destroy(R->graph);
    delete R;
    return fail(MRF_SHAPE, "recon_create: need p in {2, 3, 4, 8}, 1 <= rank_cap <= 16, 1 <= K < patch count");
  }
  const int cov1 = std::min(R->g.ppc, R->g.n1);
  R->cmax = (double)cov1 * cov1;
  const size_t Nv = R->Nv, rr = R->r, Np = R->g.Np, rc = prm->rank_cap;
  auto alloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) return nullptr;
    R->allocs.push_back(p);
    return p;
  };
  bool ok = (R->X = (cf*)alloc((size_t)L * Nv * 8)) && (R->ZG = (cf*)alloc((size_t)L * Nv * 8)) &&
            (R->res = (cf*)alloc((size_t)L * Ns * 8)) && (R->aX = (cf*)alloc(Nv * rr * 8)) &&
            (R->aU = (cf*)alloc(Nv * rr * 8)) && (R->Ya = (cf*)alloc(Nv * rr * 8)) &&
            (R->beta = (cf*)alloc(Nv * rr * 8)) && (R->U = (cf*)alloc(Np * rc * pp * 8)) &&
            (R->C = (cf*)alloc(Np * rc * (size_t)L * 8)) && (R->f = (float*)alloc(Np * rc * 4)) &&
            (R->maps = (float*)alloc(3 * Nv * 4)) && (R->rho = (float*)alloc(Nv * 4)) &&
            (R->idx = (int*)alloc(Nv * 4)) && (R->nws = alloc(nufft_ws_bytes(plan))) &&
            (R->rws = alloc(reduce_ws_bytes(L, (int)Nv, (int)rr))) &&
            (R->rws2 = alloc(reduce_ws_bytes(L, (int)Nv, (int)rr))) && (R->lws = alloc(llr_ws_bytes(R->g, (int)rc))) &&
            (R->sc = (double*)alloc(SC_N * 8)) && (R->rpart = (double*)alloc(nufft_resid_blocks(plan) * 8));
  if (ok) ok = hipHostMalloc((void**)&R->hsc, SC_N * sizeof(double), hipHostMallocDefault) == hipSuccess;
  R->res1 = R->res;
  R->rpart1 = R->rpart;
  if (!ok) {
    mrf_recon_destroy(R);
    return fail(MRF_OOM, "recon_create: device allocation failed");
  }
  for (int k = 0; k < 2 && ok; ++k)
    ok = hipStreamCreateWithFlags(&R->aux[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&R->ev_aux[k], hipEventDisableTiming) == hipSuccess;
  if (ok) ok = hipEventCreateWithFlags(&R->ev_fork, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    mrf_recon_destroy(R);
    return fail(MRF_DEVICE, "recon_create: stream or event creation failed");
  }
  *out = R;
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_destroy(mrf_recon_t R) {
  clear_error();
  if (!R) return MRF_OK;
  for (int k = 0; k < 2; ++k)
    if (R->aux[k]) hipStreamSynchronize(R->aux[k]);   // their work may still read the buffers
  for (int k = 0; k < 2; ++k) {
    if (R->aux[k]) hipStreamDestroy(R->aux[k]);
    if (R->ev_aux[k]) hipEventDestroy(R->ev_aux[k]);
  }
  if (R->ev_fork) hipEventDestroy(R->ev_fork);
  for (void* p : R->allocs) hipFree(p);
  for (void* p : R->coil_bufs) hipFree(p);
  for (void* p : R->toep_bufs) hipFree(p);
  for (auto& g : R->inj) {
    hipFree(g.rowptr); hipFree(g.col); hipFree(g.val); hipFree(g.scal);
  }
  hipFree(R->fin_ws);
  hipFree(R->fin_prm);
  if (R->hsc) hipHostFree(R->hsc);
  mrf_graph_destroy(R->graph);
  delete R;
  return MRF_OK;
}

// Multi-coil data (eq. (1)): the data term's operator becomes F_u C. Copies the maps; the residual
// buffer grows to ncoils series. The recon must be initialised again afterwards.
extern "C" mrf_status mrf_recon_set_coils(mrf_recon_t R, const mrf_c64* smaps, int ncoils, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(R, MRF_INVALID_ARG, "recon_set_coils: null handle");
  MRF_REQUIRE(!smaps || ncoils >= 1, MRF_INVALID_ARG, "recon_set_coils: ncoils must be >= 1 with sensitivity maps");
  MRF_REQUIRE(!smaps || !R->toep, MRF_NOT_SUPPORTED, "recon_set_coils: not with the Toeplitz normal operator");
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < 2; ++k) MRF_CHECK_HIP(hipStreamSynchronize(R->aux[k]));
  for (void* p : R->coil_bufs) hipFree(p);
  R->coil_bufs.clear();
  R->smaps = nullptr;
  R->ncoils = 0;
  R->res = R->res1;
  R->rpart = R->rpart1;
  R->initialised = false;
  if (!smaps) return MRF_OK;
  const size_t nmap = (size_t)ncoils * R->Nv, nres = (size_t)ncoils * R->L * R->Ns;
  const size_t npart = (size_t)ncoils * nufft_resid_blocks(R->plan);
  void *m = nullptr, *r = nullptr, *q = nullptr;
  if (hipMalloc(&m, nmap * 8) != hipSuccess || hipMalloc(&r, nres * 8) != hipSuccess ||
      hipMalloc(&q, npart * 8) != hipSuccess) {
    hipFree(m); hipFree(r); hipFree(q);
    return fail(MRF_OOM, "recon_set_coils: device allocation failed");
  }
  R->coil_bufs = {m, r, q};
  MRF_CHECK_HIP(hipMemcpyAsync(m, smaps, nmap * 8, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  R->smaps = (cf*)m;
  R->ncoils = ncoils;
  R->res = (cf*)r;
  R->rpart = (double*)q;
  return MRF_OK;
}

// The data term's gradient and value through the Toeplitz normal operator t (built from the
// plan's own trajectory); t null returns to the gridded pair. The recon must be initialised again.
extern "C" mrf_status mrf_recon_set_toeplitz(mrf_recon_t R, mrf_toeplitz_t t, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(R, MRF_INVALID_ARG, "recon_set_toeplitz: null handle");
  MRF_REQUIRE(!t || (toeplitz_n(t) == R->N && toeplitz_frames(t) == R->L), MRF_SHAPE,
              "recon_set_toeplitz: the operator's n or frame count differs from the recon's");
  MRF_REQUIRE(!t || !R->smaps, MRF_NOT_SUPPORTED, "recon_set_toeplitz: not with coil sensitivities");
  MRF_REQUIRE(!t || toeplitz_ws_bytes(t) <= nufft_ws_bytes(R->plan), MRF_SHAPE,
              "recon_set_toeplitz: the plan's workspace is smaller than the operator's");
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < 2; ++k) MRF_CHECK_HIP(hipStreamSynchronize(R->aux[k]));
  for (void* p : R->toep_bufs) hipFree(p);
  R->toep_bufs.clear();
  R->toep = nullptr;
  R->TX = R->AHb = R->AHbV = nullptr;
  R->tpart = R->bn2 = nullptr;
  R->initialised = false;
  if (!t) return MRF_OK;
  const size_t img = (size_t)R->L * R->Nv * sizeof(cf), nv = (size_t)R->Nv * R->r * sizeof(cf);
  void *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr;
  if (hipMalloc(&a, img) != hipSuccess || hipMalloc(&b, img) != hipSuccess || hipMalloc(&c, nv) != hipSuccess ||
      hipMalloc(&d, (kToepDataBlocks + 1) * sizeof(double)) != hipSuccess) {
    hipFree(a); hipFree(b); hipFree(c); hipFree(d);
    return fail(MRF_OOM, "recon_set_toeplitz: device allocation failed");
  }
  R->toep_bufs = {a, b, c, d};
  R->toep = t;
  R->TX = (cf*)a;
  R->AHb = (cf*)b;
  R->AHbV = (cf*)c;
  R->tpart = (double*)d;
  R->bn2 = R->tpart + kToepDataBlocks;
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_init(mrf_recon_t R, const mrf_c64* b, const mrf_c64* X0, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(R && b, MRF_INVALID_ARG, "recon_init: null argument");
  const auto t0 = std::chrono::steady_clock::now();
  R->b = (const cf*)b;
  R->st = mrf_recon_stats{};
  R->pending_graph = false;
  mrf_status e;
  if (X0) {
    MRF_LAUNCH("recon_copy", s, k_copy_c<<<1024, 256, 0, s>>>((const cf*)X0, R->X, (size_t)R->L * R->Nv));
    MRF_CHECK_LAUNCH();
  } else if ((e = nufft_adj_coils(R->plan, R->b, R->X, R->nws, s, R->smaps, R->ncoils))) {   // X0 = A^H b
    return e;
  }
  if (R->toep && (e = toep_prepare(R, !X0, s))) return e;
  if ((e = rebuild(R, s))) return e;
  double h[SC_N];
  if ((e = evaluate(R, s, h))) return e;
  record(R, h, true);
  record_graph(R, h);
  R->c_prev = h[SC_COST];
  R->initialised = true;
  R->st.iter_ms[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return MRF_OK;
}

namespace {

bool active(const mrf_recon_s* R) { return R->st.stop_reason == 0 && R->st.iters < R->prm.n_max; }

// Enqueues one iteration: the graph rebuild left by the previous one (if any), the gradient step
// with the projection (eqs. (15), (17)), the SVT of Q(X^n) from the previous eigen-analysis and
// the X update (eq. (23)), and the cost of X^{n+1}, whose terms are copied to the host.
mrf_status enqueue_step(mrf_recon_s* R, hipStream_t s) {
  R->t_step = std::chrono::steady_clock::now();
  const int L = R->L, Nv = R->Nv, r = R->r, rc = R->prm.rank_cap;
  const cf* V = dict_basis(R->dict);
  mrf_status e;
  // Three independent chains until the X update: the graph rebuild (aux[0]), the SVT coefficients
  // of X (aux[1]) and the data-term gradient (s), which waits for the rebuild only where it needs
  // the new graph, aX and the scalars.
  if ((e = fork(R, 2, s))) return e;
  if (R->pending_graph && (e = rebuild(R, aux_stream(R, 0, 2, s)))) return e;
  if ((e = llr_coef(R->X, R->g, L, rc, R->U, R->f, R->C, aux_stream(R, 1, 2, s)))) return e;
  if (R->toep) {
    // G V = (A^H A X) V - (A^H b) V, with A^H A X from the last cost evaluation
    if ((e = subspace_reduce(R->TX, nullptr, nullptr, V, L, Nv, r, R->aU, (cf*)R->rws, s))) return e;
    MRF_LAUNCH("recon_toep_grad", s, k_sub_c<<<ceil_div((long)Nv * r, 256), 256, 0, s>>>(R->aU, R->AHbV, (long)Nv * r));
  } else {
    if ((e = nufft_adj_coils(R->plan, R->res, R->ZG, R->nws, s, R->smaps, R->ncoils))) return e;  // G = A^H r
    if ((e = subspace_reduce(R->ZG, nullptr, nullptr, V, L, Nv, r, R->aU, (cf*)R->rws, s))) return e;  // G V
  }
  // aX = X V is current: the graph rebuild (or the initialisation) computed it from this X
  if ((e = join(R, 0, 2, s))) return e;
  if ((e = lap_apply_sub(R->graph, R->aX, R->Ya, r, s))) return e;                            // S_L(X V)
  if ((e = grad_coef(R->aX, R->aU, R->Ya, R->sc + SC_MU, R->sc + SC_LAM1, (long)Nv * r, R->beta, s))) return e;
  if (llr_xupdate_beta_ok(R->g, rc, r)) {
    // Z = beta V^H is formed inside the X update's tiles and never stored
    if ((e = join(R, 1, 2, s))) return e;
    if ((e = llr_xupdate_beta(R->beta, V, r, R->U, R->C, R->g, L, rc, R->sc + SC_KAP, 1.0, R->X, s))) return e;
    return evaluate_enqueue(R, s);
  }
  if ((e = subspace_expand(R->beta, V, L, Nv, r, R->ZG, s))) return e;                        // Z
  if ((e = join(R, 1, 2, s))) return e;
  if ((e = llr_xupdate(R->ZG, R->U, R->C, R->g, L, rc, R->sc + SC_KAP, 1.0, R->X, s))) return e;
  return evaluate_enqueue(R, s);
}

// Waits for the step's cost terms, records them and applies the stopping rule; when another
// iteration follows, the next graph rebuild is left to it (its scalars arrive with its cost).
mrf_status complete_step(mrf_recon_s* R, hipStream_t s) {
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  const double* h = R->hsc;
  if (!std::isfinite(h[SC_COST])) return fail(MRF_NONFINITE, "recon: cost is not finite");
  if (R->pending_graph) record_graph(R, h);
  R->pending_graph = false;
  R->st.iters += 1;
  record(R, h, false);
  if (R->st.iters <= MRF_MAX_ITERS)
    R->st.iter_ms[R->st.iters] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - R->t_step).count();
  const double c = h[SC_COST];
  if (R->prm.tol >= 0.0 && R->c_prev / c - 1.0 < R->prm.tol) {
    R->st.stop_reason = 1;
    return MRF_OK;
  }
  R->c_prev = c;
  R->pending_graph = R->st.iters < R->prm.n_max;   // M^{n+1}, L^{n+1}, lambda1 before the next step
  return MRF_OK;
}

}  // namespace

extern "C" mrf_status mrf_recon_iterate(mrf_recon_t R, int n, int* stopped, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(R && R->initialised, MRF_INVALID_ARG, "recon_iterate: call mrf_recon_init first");
  MRF_REQUIRE(n >= 0, MRF_INVALID_ARG, "recon_iterate: n must be >= 0");
  mrf_status e;
  for (int it = 0; it < n && active(R); ++it) {
    if ((e = enqueue_step(R, s))) return e;
    if ((e = complete_step(R, s))) return e;
  }
  if (stopped) *stopped = !active(R);
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_set_serial(mrf_recon_t R, int serial) {
  clear_error();
  MRF_REQUIRE(R, MRF_INVALID_ARG, "recon_set_serial: null handle");
  R->prm.serial = serial;
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_batched(int nslices, const mrf_recon_t* Rs, const hipStream_t* streams, int n,
                                        int* n_active) {
  clear_error();
  MRF_REQUIRE(nslices >= 1 && Rs && streams && n >= 0, MRF_INVALID_ARG, "recon_batched: bad argument");
  for (int i = 0; i < nslices; ++i)
    MRF_REQUIRE(Rs[i] && Rs[i]->initialised, MRF_INVALID_ARG, "recon_batched: every slice needs mrf_recon_init");
  mrf_status e;
  for (int it = 0; it < n; ++it) {
    bool any = false;
    for (int i = 0; i < nslices; ++i)
      if (active(Rs[i])) {
        if ((e = enqueue_step(Rs[i], streams[i]))) return e;
        any = true;
      }
    if (!any) break;
    for (int i = 0; i < nslices; ++i)
      if (Rs[i]->st.iters < Rs[i]->prm.n_max && Rs[i]->st.stop_reason == 0 && (e = complete_step(Rs[i], streams[i])))
        return e;
  }
  if (n_active) {
    int k = 0;
    for (int i = 0; i < nslices; ++i) k += active(Rs[i]);
    *n_active = k;
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_finish(mrf_recon_t R, mrf_c64* X_out, float* maps, int32_t* idx, float* rho,
                                       hipStream_t s) {
  clear_error();
  MRF_REQUIRE(R && R->initialised, MRF_INVALID_ARG, "recon_finish: call mrf_recon_init first");
  mrf_status e;
  const cf* V = dict_basis(R->dict);
  const int Nv = R->Nv;
  if (R->fin_mode == MRF_MATCH_SUBSPACE || R->fin_mode == MRF_MATCH_LEARNED)
    if ((e = subspace_reduce(R->X, nullptr, nullptr, V, R->L, Nv, R->r, R->aX, (cf*)R->rws, s))) return e;
  if (R->fin_mode == MRF_MATCH_SUBSPACE) {
    if ((e = match_subspace(R->dict, R->aX, Nv, R->idx, R->rho, nullptr, nullptr, s))) return e;
    if ((e = maps_from_match(R->dict, R->idx, R->rho, Nv, R->maps, s))) return e;
  } else if (R->fin_mode == MRF_MATCH_LEARNED) {
    int nfb = 0;
    if ((e = mrf_mlp_match(R->fin_mlp, R->dict, (const mrf_c64*)R->aX, Nv, 0, R->fin_theta, R->idx, R->fin_prm, R->rho,
                           nullptr, nullptr, &nfb, R->fin_ws, R->fin_ws_bytes, s)))
      return e;
    MRF_LAUNCH("recon_maps", s, k_maps_params<<<ceil_div(Nv, 256), 256, 0, s>>>(R->fin_prm, 2, R->rho, Nv, R->maps));
  } else {
    // X^ to voxel-major time courses in the gradient buffer (free once the iterations are done)
    if ((e = mrf_frames_to_voxels((const mrf_c64*)R->X, R->L, Nv, (mrf_c64*)R->ZG, s))) return e;
    if ((e = mrf_dict_match(R->dict, (const mrf_c64*)R->ZG, Nv, (mrf_match_mode)R->fin_mode, R->idx, R->rho, nullptr,
                            R->fin_prm, nullptr, R->fin_ws, R->fin_ws_bytes, s)))
      return e;
    MRF_LAUNCH("recon_maps", s,
               k_maps_params<<<ceil_div(Nv, 256), 256, 0, s>>>(R->fin_prm, R->dict->nparam, R->rho, Nv, R->maps));
  }
  MRF_CHECK_LAUNCH();
  if (X_out) MRF_CHECK_HIP(hipMemcpyAsync(X_out, R->X, (size_t)R->L * R->Nv * 8, hipMemcpyDeviceToDevice, s));
  if (maps) MRF_CHECK_HIP(hipMemcpyAsync(maps, R->maps, (size_t)3 * R->Nv * 4, hipMemcpyDeviceToDevice, s));
  if (idx) MRF_CHECK_HIP(hipMemcpyAsync(idx, R->idx, (size_t)R->Nv * 4, hipMemcpyDeviceToDevice, s));
  if (rho) MRF_CHECK_HIP(hipMemcpyAsync(rho, R->rho, (size_t)R->Nv * 4, hipMemcpyDeviceToDevice, s));
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_inject_graph(mrf_recon_t R, int k, int nnz, const int* rowptr, const int* col,
                                             const float* val, double sigma2, double lmax) {
  clear_error();
  MRF_REQUIRE(R && rowptr && col && val, MRF_INVALID_ARG, "recon_inject_graph: null argument");
  MRF_REQUIRE(k >= 0 && k <= MRF_MAX_ITERS, MRF_INVALID_ARG, "recon_inject_graph: graph number out of range");
  const int Np = R->g.Np;
  MRF_REQUIRE(nnz >= Np && (size_t)nnz <= graph_capacity(R->graph), MRF_SHAPE,
              "recon_inject_graph: nnz must lie between the patch count and the graph's capacity");
  MRF_REQUIRE(rowptr[0] == 0 && rowptr[Np] == nnz, MRF_INVALID_ARG, "recon_inject_graph: rowptr must run from 0 to nnz");
  for (int i = 0; i < Np; ++i) {
    MRF_REQUIRE(rowptr[i + 1] > rowptr[i], MRF_INVALID_ARG, "recon_inject_graph: every row needs its diagonal");
    bool diag = false;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      MRF_REQUIRE(col[e] >= 0 && col[e] < Np && (e == rowptr[i] || col[e] > col[e - 1]), MRF_INVALID_ARG,
                  "recon_inject_graph: columns must be in range and ascending within a row");
      diag |= col[e] == i;
    }
    MRF_REQUIRE(diag, MRF_INVALID_ARG, "recon_inject_graph: every row needs its diagonal");
  }
  MRF_REQUIRE(sigma2 > 0.0 && lmax >= 0.0, MRF_INVALID_ARG, "recon_inject_graph: need sigma2 > 0 and lmax >= 0");
  mrf_recon_s::Injected g{k, nnz, nullptr, nullptr, nullptr, nullptr};
  const double scal[4] = {sigma2, lmax, (double)nnz, 0.0};
  bool ok = hipMalloc(&g.rowptr, (size_t)(Np + 1) * 4) == hipSuccess && hipMalloc(&g.col, (size_t)nnz * 4) == hipSuccess &&
            hipMalloc(&g.val, (size_t)nnz * 4) == hipSuccess && hipMalloc(&g.scal, sizeof scal) == hipSuccess;
  ok = ok && hipMemcpy(g.rowptr, rowptr, (size_t)(Np + 1) * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(g.col, col, (size_t)nnz * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(g.val, val, (size_t)nnz * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(g.scal, scal, sizeof scal, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    hipFree(g.rowptr); hipFree(g.col); hipFree(g.val); hipFree(g.scal);
    return fail(MRF_OOM, "recon_inject_graph: device allocation or copy failed");
  }
  for (auto& old : R->inj)
    if (old.k == k) {
      hipFree(old.rowptr); hipFree(old.col); hipFree(old.val); hipFree(old.scal);
      old = g;
      return MRF_OK;
    }
  R->inj.push_back(g);
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_set_final_match(mrf_recon_t R, mrf_match_mode mode, mrf_mlp_t mlp, float theta) {
  clear_error();
  MRF_REQUIRE(R, MRF_INVALID_ARG, "recon_set_final_match: null handle");
  MRF_REQUIRE(mode == MRF_MATCH_SUBSPACE || mode == MRF_MATCH_FP32 || mode == MRF_MATCH_BF16_RERANK4 ||
                  mode == MRF_MATCH_FP8_RERANK4 || mode == MRF_MATCH_BF16X3_RERANK || mode == MRF_MATCH_LEARNED,
              MRF_INVALID_ARG, "recon_set_final_match: unknown mode");
  MRF_REQUIRE(mode != MRF_MATCH_LEARNED || mlp, MRF_INVALID_ARG, "recon_set_final_match: the learned mode needs an MLP");
  MRF_REQUIRE(theta == theta, MRF_INVALID_ARG, "recon_set_final_match: theta is NaN");
  size_t ws = 0, prm = 0;
  if (mode == MRF_MATCH_LEARNED) {
    mrf_status e = mrf_mlp_match_workspace_size(mlp, R->Nv, &ws);
    if (e) return e;
    prm = (size_t)R->Nv * 2 * sizeof(float);
  } else if (mode != MRF_MATCH_SUBSPACE) {
    mrf_status e = mrf_dict_match_workspace_size(R->dict, R->Nv, mode, &ws);
    if (e) return e;
    prm = (size_t)R->Nv * R->dict->nparam * sizeof(float);
  }
  MRF_CHECK_HIP(hipDeviceSynchronize());   // the previous buffers may still be in use
  hipFree(R->fin_ws);
  hipFree(R->fin_prm);
  R->fin_ws = nullptr;
  R->fin_prm = nullptr;
  R->fin_ws_bytes = 0;
  R->fin_mode = MRF_MATCH_SUBSPACE;
  if ((ws && hipMalloc(&R->fin_ws, ws) != hipSuccess) || (prm && hipMalloc((void**)&R->fin_prm, prm) != hipSuccess)) {
    hipFree(R->fin_ws);
    R->fin_ws = nullptr;
    return fail(MRF_OOM, "recon_set_final_match: device allocation failed");
  }
  R->fin_ws_bytes = ws;
  R->fin_mode = mode;
  R->fin_mlp = mlp;
  R->fin_theta = theta;
  return MRF_OK;
}

namespace {
// checkpoint: a header (sizes for the check on load, stopping state, statistics), then the arrays
struct CkptHeader {
  uint64_t magic;
  int version, N, L, Ns, Np, rcap, pp, r, pending, ncoils;   // ncoils 0: single coil, no maps
  int toeplitz, pad;                                          // 1: saved in the Toeplitz mode
  double c_prev;
  mrf_recon_stats st;
};
constexpr uint64_t kCkptMagic = 0x4d52464c4c52636bull;   // "MRFLLRck"
size_t ck_al(size_t b) { return (b + 255) & ~(size_t)255; }
struct CkptLayout {
  size_t x, res, u, f, sc, total;
};
CkptLayout ckpt_layout(const mrf_recon_s* R) {
  CkptLayout c;
  const size_t pp = (size_t)R->prm.p * R->prm.p, np = R->g.Np, rc = R->prm.rank_cap;
  c.x = ck_al(sizeof(CkptHeader));
  c.res = c.x + ck_al((size_t)R->L * R->Nv * 8);
  c.u = c.res + ck_al((size_t)std::max(1, R->ncoils) * R->L * R->Ns * 8);
  c.f = c.u + ck_al(np * rc * pp * 8);
  c.sc = c.f + ck_al(np * rc * 4);
  c.total = c.sc + ck_al(SC_N * 8);
  return c;
}
}  // namespace

extern "C" mrf_status mrf_recon_checkpoint_bytes(mrf_recon_t R, size_t* bytes) {
  clear_error();
  MRF_REQUIRE(R && bytes, MRF_INVALID_ARG, "recon_checkpoint_bytes: null argument");
  *bytes = ckpt_layout(R).total;
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_checkpoint_save(mrf_recon_t R, void* buf, size_t bytes, hipStream_t s) {
  clear_error();
  MRF_REQUIRE(R && buf, MRF_INVALID_ARG, "recon_checkpoint_save: null argument");
  MRF_REQUIRE(R->initialised, MRF_INVALID_ARG, "recon_checkpoint_save: call mrf_recon_init first");
  const CkptLayout c = ckpt_layout(R);
  MRF_REQUIRE(bytes >= c.total, MRF_WORKSPACE, "recon_checkpoint_save: buffer smaller than mrf_recon_checkpoint_bytes");
  CkptHeader h{};
  h.magic = kCkptMagic;
  h.version = 2;
  h.N = R->N; h.L = R->L; h.Ns = R->Ns; h.Np = R->g.Np; h.rcap = R->prm.rank_cap; h.pp = R->prm.p * R->prm.p;
  h.r = R->r;
  h.pending = R->pending_graph ? 1 : 0;
  h.ncoils = R->ncoils;
  h.toeplitz = R->toep ? 1 : 0;
  h.c_prev = R->c_prev;
  h.st = R->st;
  char* o = (char*)buf;
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.x, R->X, (size_t)R->L * R->Nv * 8, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.res, R->res, (size_t)std::max(1, R->ncoils) * R->L * R->Ns * 8,
                               hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.u, R->U, (size_t)h.Np * h.rcap * h.pp * 8, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.f, R->f, (size_t)h.Np * h.rcap * 4, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(o + c.sc, R->sc, SC_N * 8, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  MRF_CHECK_HIP(hipMemcpy(o, &h, sizeof h, hipMemcpyDefault));
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_checkpoint_load(mrf_recon_t R, const mrf_c64* b, const void* buf, size_t bytes,
                                                hipStream_t s) {
  clear_error();
  MRF_REQUIRE(R && b && buf, MRF_INVALID_ARG, "recon_checkpoint_load: null argument");
  const CkptLayout c = ckpt_layout(R);
  MRF_REQUIRE(bytes >= c.total, MRF_WORKSPACE, "recon_checkpoint_load: buffer smaller than mrf_recon_checkpoint_bytes");
  CkptHeader h{};
  const char* o = (const char*)buf;
  MRF_CHECK_HIP(hipMemcpy(&h, o, sizeof h, hipMemcpyDefault));
  MRF_REQUIRE(h.magic == kCkptMagic && h.version == 2, MRF_INVALID_ARG, "recon_checkpoint_load: not a checkpoint");
  MRF_REQUIRE(h.N == R->N && h.L == R->L && h.Ns == R->Ns && h.Np == R->g.Np && h.rcap == R->prm.rank_cap &&
                  h.pp == R->prm.p * R->prm.p && h.r == R->r && h.ncoils == R->ncoils &&
                  h.toeplitz == (R->toep ? 1 : 0),
              MRF_SHAPE, "recon_checkpoint_load: the checkpoint's sizes differ from this recon's");
  MRF_CHECK_HIP(hipMemcpyAsync(R->X, o + c.x, (size_t)R->L * R->Nv * 8, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(R->res, o + c.res, (size_t)std::max(1, R->ncoils) * R->L * R->Ns * 8,
                               hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(R->U, o + c.u, (size_t)h.Np * h.rcap * h.pp * 8, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(R->f, o + c.f, (size_t)h.Np * h.rcap * 4, hipMemcpyDefault, s));
  MRF_CHECK_HIP(hipMemcpyAsync(R->sc, o + c.sc, SC_N * 8, hipMemcpyDefault, s));
  R->b = (const cf*)b;
  R->st = h.st;
  R->c_prev = h.c_prev;
  R->pending_graph = h.pending != 0;
  R->initialised = true;
  if (R->toep) {
    // A^H b, (A^H b) V, ||b||^2 and A^H A X are functions of b and the restored X: recomputed
    mrf_status e = toep_prepare(R, false, s);
    if (!e) e = toeplitz_apply(R->toep, R->X, R->TX, R->nws, s);
    if (e) return e;
  }
  if (!R->pending_graph && active(R)) {
    // saved right after the initialisation: its graph is rebuilt from X^0 (the same deterministic
    // kernels on the same data give the same graph, lambda1 and mu); the statistics already hold it
    mrf_status e = rebuild(R, s);
    if (e) return e;
  }
  MRF_CHECK_HIP(hipStreamSynchronize(s));
  return MRF_OK;
}

extern "C" mrf_status mrf_recon_get_stats(mrf_recon_t R, mrf_recon_stats* out) {
  clear_error();
  MRF_REQUIRE(R && out, MRF_INVALID_ARG, "recon_get_stats: null argument");
  *out = R->st;
  return MRF_OK;
}

extern "C" mrf_status mrf_recon(mrf_recon_t R, const mrf_c64* b, const mrf_c64* X0, mrf_c64* X_out, float* maps,
                                int32_t* idx, float* rho, mrf_recon_stats* stats, hipStream_t s) {
  mrf_status e = mrf_recon_init(R, b, X0, s);
  if (e) return e;
  int stopped = 0;
  if ((e = mrf_recon_iterate(R, R->prm.n_max, &stopped, s))) return e;
  if ((e = mrf_recon_finish(R, X_out, maps, idx, rho, s))) return e;
  if (stats) *stats = R->st;
  return MRF_OK;
}
