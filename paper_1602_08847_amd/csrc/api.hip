// Context, iteration driver and C ABI of libmuffin (declarations and contracts in include/muffin.h).
//
// One iteration of Algorithm 1 (Sec. 3) is enqueued as four phases on the context's stream:
//   1. spatial adjoint   a = W_s^dagger (omega u), by Horner over the scales (eq. (adjointspat));
//   2. gradient          q = w H^dagger H x - b + mu_s a, three FFT passes (eq. (grad));
//   3. spectral step     fused per-pixel kernel: t, x~, d, V update, x relaxation;
//   4. spatial dual step analysis of d scale by scale, fused with sat and relaxation of U
//                        (eq. (anaylsespat) and eq. (updatenode)).
// Phases 1-2 are per channel and phase 3 per pixel: the two synchronisation points play the
// part of the paper's master/node exchanges.  After the first call the iteration is replayed
// from a captured HIP graph.
#include "common.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace mf {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

int fft_init_attrs(int N);
int atrous_init_attrs();
int spectral_init_attrs(int L);
int launch_power_spectrum(const float2* Hhat_T, float* P_T, const float* chan_w, long long per_ch, int nch,
                          float scale, hipStream_t st);
int launch_clamp_pos(float* x, long long n, hipStream_t st);
int launch_scale_channels(float* x, const float* chan_w, long long npix, int nch, hipStream_t st);
int cnn_warm_input(const float* Y, const float* scale, float* out, int N, int L, hipStream_t st);
int launch_psf_lobe(const float* psf, float* out, int N, int L, int radius, hipStream_t st);
}  // namespace mf

using namespace mf;

struct muffin_ctx {
  muffin_params p{};
  std::vector<float> chan_w_host;
  int N = 0, L = 0, J = 0, gen = 2;
  long long npix = 0, cube = 0;
  FftGeom g;
  int device = 0;
  hipStream_t user = nullptr, st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, e0 = nullptr, e1 = nullptr;
  hipEvent_t ph[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t kev[16] = {};  // per-launch timing marks (profiling only)
  double kms_an = 0, kms_ad = 0;  // summed per-launch times of the last profiled iteration
  int kn_an = 0, kn_ad = 0;
  float *X = nullptr, *U = nullptr, *V = nullptr, *D = nullptr, *Q = nullptr, *B = nullptr, *Y = nullptr;
  float *cA = nullptr, *cB = nullptr, *cT = nullptr;
  float2* S = nullptr;
  float2* Hhat_T = nullptr;
  float* P_T = nullptr;
  float2* tw = nullptr;
  float2 *twL = nullptr, *csL = nullptr;
  float *W = nullptr, *WT = nullptr;
  float* chan_w = nullptr;
  float* psf_lobe = nullptr;  // [L] sum of each PSF over the 9 x 9 window at its origin
  double* partial = nullptr;
  double* dres = nullptr;  // device scalars
  double tau = 0, sigma = 1, rho = 1, beta = 0, K2 = 0, Ws2 = 0, delta = 0;
  float omega_c = 1.f;
  long long iter = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

namespace {

struct StreamScope {
  // Orders the library stream after the caller's stream on entry, and the caller's stream after
  // the library stream on exit.
  muffin_ctx* c;
  bool ok = true;
  explicit StreamScope(muffin_ctx* c_) : c(c_) {
    ok = hipEventRecord(c->ev_in, c->user) == hipSuccess && hipStreamWaitEvent(c->st, c->ev_in, 0) == hipSuccess;
  }
  ~StreamScope() {
    if (hipEventRecord(c->ev_out, c->st) == hipSuccess) (void)hipStreamWaitEvent(c->user, c->ev_out, 0);
  }
};

template <typename T>
int dalloc(T** p, size_t n) {
  if (hipMalloc((void**)p, sizeof(T) * (n ? n : 1)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation failed (" + std::to_string(sizeof(T) * n) + " bytes)");
    return MUFFIN_ENOMEM;
  }
  return MUFFIN_OK;
}

PlaneRef pref(const float* p, long long cs) { return PlaneRef{p, cs}; }
PlaneOut pout(float* p, long long cs) { return PlaneOut{p, cs}; }

int validate(const muffin_params* p) {
  if (!p) return set_error("params is NULL"), MUFFIN_EINVAL;
  if (!fft_supported(p->N)) return set_error("N must be 2^a or 3*2^a with 8 <= N <= 1024"), MUFFIN_EINVAL;
  if (p->L < 1 || p->L > 512) return set_error("L must be in [1, 512]"), MUFFIN_EINVAL;
  if (p->J < 1 || p->J > 6) return set_error("J must be in [1, 6]"), MUFFIN_EINVAL;
  if (p->iuwt_gen != 1 && p->iuwt_gen != 2) return set_error("iuwt_gen must be 1 or 2"), MUFFIN_EINVAL;
  if (p->penalize_coarse != 0 && p->penalize_coarse != 1)
    return set_error("penalize_coarse must be 0 or 1"), MUFFIN_EINVAL;
  if (!(p->mu_s >= 0) || !(p->mu_lambda >= 0) || !std::isfinite(p->mu_s) || !std::isfinite(p->mu_lambda))
    return set_error("mu_s and mu_lambda must be finite and >= 0"), MUFFIN_EINVAL;
  if (!(p->sigma > 0) || !std::isfinite(p->sigma)) return set_error("sigma must be > 0"), MUFFIN_EINVAL;
  if (!(p->rho > 0) || !std::isfinite(p->rho)) return set_error("rho must be > 0"), MUFFIN_EINVAL;
  if (!std::isfinite(p->tau)) return set_error("tau must be finite"), MUFFIN_EINVAL;
  if (p->chan_weight) {
    for (int l = 0; l < p->L; ++l)
      if (!(p->chan_weight[l] > 0) || !std::isfinite(p->chan_weight[l]))
        return set_error("chan_weight entries must be finite and > 0"), MUFFIN_EINVAL;
  }
  return MUFFIN_OK;
}

// ---------------------------------------------------------------- phases
// Spatial adjoint of omega-weighted U; returns the buffer holding a = W_s^dagger (omega u).
int enqueue_adjoint(muffin_ctx* c, const float* Ubase, long long ucs, float omega_c, const float** result,
                    bool timed = false) {
  const int J = c->J;
  const long long np = c->npix;
  const float* a = Ubase + (long long)J * np;  // coarse plane
  long long acs = ucs;
  float* bufs[2] = {c->cA, c->cB};
  int nb = 0;
  if (omega_c != 1.f) {
    MF_TRY(launch_pointwise(PT_COPY, c->N, c->L, pref(a, acs), PlaneRef{}, pout(c->cA, np), omega_c, 1.f, nullptr,
                            nullptr, c->st));
    a = c->cA;
    acs = np;
    nb = 1;
  }
  for (int j = J - 1; j >= 0; --j) {
    const float* uj = Ubase + (long long)j * np;
    float* dst = bufs[nb];
    if (c->gen == 2 && atrous_double_fits(c->N, j, nullptr, nullptr)) {
      if (timed) MF_HIP(hipEventRecord(c->kev[2 * j], c->st));
      MF_TRY(launch_atrous(DB_ADJOINT, c->N, c->L, j, pref(uj, ucs), pref(a, acs), PlaneRef{}, pout(dst, np),
                           PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
      if (timed) MF_HIP(hipEventRecord(c->kev[2 * j + 1], c->st));
    } else {
      const float* sub = uj;
      long long scs = ucs;
      if (c->gen == 2) {
        MF_TRY(launch_atrous(SM_SMOOTH, c->N, c->L, j, pref(uj, ucs), PlaneRef{}, PlaneRef{}, pout(c->cT, np),
                             PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
        sub = c->cT;
        scs = np;
      }
      MF_TRY(launch_atrous(SM_SUBADD, c->N, c->L, j, pref(a, acs), pref(sub, scs), pref(uj, ucs), pout(dst, np),
                           PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
    }
    a = dst;
    acs = np;
    nb ^= 1;
  }
  *result = a;
  return MUFFIN_OK;
}

// Analysis of the channel images in (stride np) fused with the spatial dual step on U.
int enqueue_dual_update(muffin_ctx* c, const float* in, bool timed = false) {
  const int J = c->J;
  const long long np = c->npix, ucs = (long long)(J + 1) * np;
  const float coef = (float)(c->sigma * c->p.mu_s);
  const float rho = (float)c->rho;
  const float* cur = in;
  float* bufs[2] = {c->cA, c->cB};
  for (int j = 0; j < J; ++j) {
    float* nxt = bufs[j & 1];
    float* uj = c->U + (long long)j * np;
    if (c->gen == 1) {
      MF_TRY(launch_atrous(SM_DETAIL1, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(uj, ucs),
                           pout(nxt, np), coef, rho, nullptr, nullptr, c->st));
    } else if (atrous_double_fits(c->N, j, nullptr, nullptr)) {
      if (timed) MF_HIP(hipEventRecord(c->kev[2 * j], c->st));
      MF_TRY(launch_atrous(DB_ANALYSIS, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(uj, ucs),
                           pout(nxt, np), coef, rho, nullptr, nullptr, c->st));
      if (timed) MF_HIP(hipEventRecord(c->kev[2 * j + 1], c->st));
    } else {
      MF_TRY(launch_atrous(SM_SMOOTH, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(nxt, np),
                           PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
      MF_TRY(launch_atrous(SM_DETAIL, c->N, c->L, j, pref(nxt, np), PlaneRef{}, pref(cur, np), pout(uj, ucs),
                           PlaneOut{}, coef, rho, nullptr, nullptr, c->st));
    }
    cur = nxt;
  }
  MF_TRY(launch_pointwise(PT_COARSE, c->N, c->L, pref(cur, np), PlaneRef{}, pout(c->U + (long long)J * np, ucs),
                          coef * c->omega_c, rho, nullptr, nullptr, c->st));
  return MUFFIN_OK;
}

int enqueue_gradient(muffin_ctx* c, const float* x, float* out, const float* s, float s_scale) {
  MF_TRY(launch_rows_r2c(x, c->S, c->L, c->g, c->tw, false, c->st));
  MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, COL_REAL, c->P_T, nullptr, 1.f, nullptr, c->st));
  MF_TRY(launch_rows_c2r(c->S, c->L, c->g, c->tw, EPI_GRAD, out, c->B, s, s_scale, nullptr, nullptr, nullptr,
                         nullptr, c->st));
  return MUFFIN_OK;
}

int enqueue_spectral(muffin_ctx* c) {
  SpectralArgs a;
  a.X = c->X;
  a.Q = c->Q;
  a.V = c->V;
  a.D = c->D;
  a.W = c->W;
  a.WT = c->WT;
  a.twL = c->twL;
  a.csL = c->csL;
  a.npix = c->npix;
  a.L = c->L;
  a.use_fft = spectral_has_fft(c->L) ? 1 : 0;
  a.tau = (float)c->tau;
  a.mu_l = (float)c->p.mu_lambda;
  a.smu_l = (float)(c->sigma * c->p.mu_lambda);
  a.rho = (float)c->rho;
  return launch_spectral_step(a, c->st);
}

// With marks, phase boundaries are recorded in marks[0..4] and, for the second-generation
// transform, each scale's fused adjoint (marks pass 1) or analysis launch is bracketed in kev.
int enqueue_iteration(muffin_ctx* c, hipEvent_t* marks, int timed_family = 0) {
  const long long ucs = (long long)(c->J + 1) * c->npix;
  if (marks) MF_HIP(hipEventRecord(marks[0], c->st));
  const float* s = nullptr;
  MF_TRY(enqueue_adjoint(c, c->U, ucs, c->omega_c, &s, timed_family == 1));
  if (marks) MF_HIP(hipEventRecord(marks[1], c->st));
  MF_TRY(enqueue_gradient(c, c->X, c->Q, s, (float)c->p.mu_s));
  if (marks) MF_HIP(hipEventRecord(marks[2], c->st));
  MF_TRY(enqueue_spectral(c));
  if (marks) MF_HIP(hipEventRecord(marks[3], c->st));
  MF_TRY(enqueue_dual_update(c, c->D, timed_family == 2));
  if (marks) MF_HIP(hipEventRecord(marks[4], c->st));
  return MUFFIN_OK;
}

// Objective terms at X into dres[1..3] (data, spatial l1 unweighted by mu_s, spectral l1).
int enqueue_objective(muffin_ctx* c) {
  const long long np = c->npix;
  MF_HIP(hipMemsetAsync(c->dres, 0, sizeof(double) * 4, c->st));
  int nb = 0;
  MF_TRY(launch_rows_r2c(c->X, c->S, c->L, c->g, c->tw, false, c->st));
  MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, COL_CPLX, nullptr, c->Hhat_T, 1.f / ((float)c->N * c->N), nullptr,
                     c->st));
  MF_TRY(launch_rows_c2r(c->S, c->L, c->g, c->tw, EPI_RESID, nullptr, nullptr, nullptr, 0.f, c->Y, c->chan_w,
                         c->partial, &nb, c->st));
  MF_TRY(launch_reduce_sum(c->partial, nb, c->dres + 1, 0, c->st));
  const float* cur = c->X;
  float* bufs[2] = {c->cA, c->cB};
  for (int j = 0; j < c->J; ++j) {
    float* nxt = bufs[j & 1];
    MF_TRY(launch_atrous(SM_SMOOTH, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(nxt, np),
                         PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
    if (c->gen == 2)
      MF_TRY(launch_atrous(SM_DETAIL_ABS, c->N, c->L, j, pref(nxt, np), PlaneRef{}, pref(cur, np), PlaneOut{},
                           PlaneOut{}, 0.f, 1.f, c->partial, &nb, c->st));
    else
      MF_TRY(launch_pointwise(PT_ABS_DIFF, c->N, c->L, pref(nxt, np), pref(cur, np), PlaneOut{}, 0.f, 1.f,
                              c->partial, &nb, c->st));
    MF_TRY(launch_reduce_sum(c->partial, nb, c->dres + 2, 1, c->st));
    cur = nxt;
  }
  if (c->omega_c != 0.f) {
    MF_TRY(launch_pointwise(PT_ABS, c->N, c->L, pref(cur, np), PlaneRef{}, PlaneOut{}, 0.f, 1.f, c->partial, &nb,
                            c->st));
    MF_TRY(launch_reduce_sum(c->partial, nb, c->dres + 2, 1, c->st));
  }
  MF_TRY(launch_dct_abs(c->X, c->WT, np, c->L, c->partial, &nb, c->st));
  MF_TRY(launch_reduce_sum(c->partial, nb, c->dres + 3, 0, c->st));
  return MUFFIN_OK;
}

void destroy(muffin_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  void* bufs[] = {c->X, c->U, c->V, c->D, c->Q, c->B, c->Y, c->cA, c->cB, c->cT, c->S, c->Hhat_T, c->P_T,
                  c->tw, c->twL, c->csL, c->W, c->WT, c->chan_w, c->psf_lobe, c->partial, c->dres};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  hipEvent_t evs[] = {c->ev_in, c->ev_out, c->e0, c->e1, c->ph[0], c->ph[1], c->ph[2], c->ph[3], c->ph[4]};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->kev)
    if (e) (void)hipEventDestroy(e);
  if (c->st) (void)hipStreamDestroy(c->st);
  delete c;
}

int copy_in(float* dst, const float* src, size_t n, int on_device, hipStream_t st) {
  MF_HIP(hipMemcpyAsync(dst, src, n * sizeof(float), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if (!on_device) MF_HIP(hipStreamSynchronize(st));
  return MUFFIN_OK;
}

int copy_out(float* dst, const float* src, size_t n, int on_device, hipStream_t st) {
  MF_HIP(hipMemcpyAsync(dst, src, n * sizeof(float), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  if (!on_device) MF_HIP(hipStreamSynchronize(st));
  return MUFFIN_OK;
}

int init_impl(muffin_ctx* c, const muffin_params* p, const float* dirty, const float* psf, int on_device) {
  c->p = *p;
  c->N = p->N;
  c->L = p->L;
  c->J = p->J;
  c->gen = p->iuwt_gen;
  c->npix = (long long)p->N * p->N;
  c->cube = c->npix * p->L;
  c->g = fft_geom(p->N);
  c->omega_c = p->penalize_coarse ? 1.f : 0.f;
  c->sigma = p->sigma;
  c->rho = p->rho;
  if (p->chan_weight) c->chan_w_host.assign(p->chan_weight, p->chan_weight + p->L);
  c->p.chan_weight = nullptr;
  MF_HIP(hipGetDevice(&c->device));
  MF_HIP(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking));
  for (hipEvent_t* e : {&c->ev_in, &c->ev_out}) MF_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  for (hipEvent_t* e : {&c->e0, &c->e1, &c->ph[0], &c->ph[1], &c->ph[2], &c->ph[3], &c->ph[4]})
    MF_HIP(hipEventCreate(e));
  for (auto& e : c->kev) MF_HIP(hipEventCreate(&e));
  MF_TRY(fft_init_attrs(c->N));
  MF_TRY(atrous_init_attrs());
  MF_TRY(spectral_init_attrs(c->L));

  const long long cube = c->cube;
  const long long spec = (long long)c->L * c->N * c->g.pitch;
  MF_TRY(dalloc(&c->X, cube));
  MF_TRY(dalloc(&c->U, cube * (c->J + 1)));
  MF_TRY(dalloc(&c->V, cube));
  MF_TRY(dalloc(&c->D, cube));
  MF_TRY(dalloc(&c->Q, cube));
  MF_TRY(dalloc(&c->B, cube));
  MF_TRY(dalloc(&c->Y, cube));
  MF_TRY(dalloc(&c->cA, cube));
  MF_TRY(dalloc(&c->cB, cube));
  MF_TRY(dalloc(&c->cT, cube));
  MF_TRY(dalloc(&c->S, spec));
  MF_TRY(dalloc(&c->Hhat_T, spec));
  MF_TRY(dalloc(&c->P_T, spec));
  MF_TRY(dalloc(&c->tw, c->N));
  MF_TRY(dalloc(&c->twL, c->L));
  MF_TRY(dalloc(&c->csL, c->L));
  MF_TRY(dalloc(&c->W, (long long)c->L * c->L));
  MF_TRY(dalloc(&c->WT, (long long)c->L * c->L));
  MF_TRY(dalloc(&c->partial, kMaxPartials));
  MF_TRY(dalloc(&c->dres, 16));
  MF_TRY(dalloc(&c->psf_lobe, c->L));
  if (!c->chan_w_host.empty()) MF_TRY(dalloc(&c->chan_w, c->L));

  StreamScope scope(c);
  if (!scope.ok) return set_error("stream ordering failed"), MUFFIN_EHIP;
  hipStream_t st = c->st;
  MF_HIP(hipMemsetAsync(c->S, 0, sizeof(float2) * spec, st));
  MF_HIP(hipMemsetAsync(c->dres, 0, sizeof(double) * 16, st));
  MF_TRY(copy_in(c->Y, dirty, cube, on_device, st));
  MF_TRY(copy_in(c->cT, psf, cube, on_device, st));
  if (c->chan_w) MF_TRY(copy_in(c->chan_w, c->chan_w_host.data(), c->L, 0, st));
  {
    auto tw = fft_twiddles(c->N);
    MF_HIP(hipMemcpyAsync(c->tw, tw.data(), sizeof(float2) * c->N, hipMemcpyHostToDevice, st));
    auto twl = fft_twiddles(c->L);
    std::vector<float2> cs(c->L);
    for (int k = 0; k < c->L; ++k) {
      const double th = M_PI * k / (2.0 * c->L);
      cs[k] = make_float2((float)std::cos(th), (float)std::sin(th));
    }
    MF_HIP(hipMemcpyAsync(c->twL, twl.data(), sizeof(float2) * c->L, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(c->csL, cs.data(), sizeof(float2) * c->L, hipMemcpyHostToDevice, st));
    std::vector<float> W((size_t)c->L * c->L), WT((size_t)c->L * c->L);
    for (int l = 0; l < c->L; ++l)
      for (int k = 0; k < c->L; ++k) {
        const double s = (k == 0) ? std::sqrt(1.0 / c->L) : std::sqrt(2.0 / c->L);
        const double v = s * std::cos(M_PI * (2.0 * l + 1.0) * k / (2.0 * c->L));
        W[(size_t)l * c->L + k] = (float)v;
        WT[(size_t)k * c->L + l] = (float)v;
      }
    MF_HIP(hipMemcpyAsync(c->W, W.data(), sizeof(float) * W.size(), hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(c->WT, WT.data(), sizeof(float) * WT.size(), hipMemcpyHostToDevice, st));
    MF_HIP(hipStreamSynchronize(st));
  }
  // non-finite inputs
  MF_TRY(launch_count_nonfinite(c->Y, cube, c->partial, c->dres + 0, st));
  MF_TRY(launch_count_nonfinite(c->cT, cube, c->partial, c->dres + 0, st));
  double bad = 0;
  MF_HIP(hipMemcpyAsync(&bad, c->dres, sizeof(double), hipMemcpyDeviceToHost, st));
  MF_HIP(hipStreamSynchronize(st));
  if (bad != 0) return set_error("NaN or Inf in dirty or psf"), MUFFIN_ENONFINITE;

  MF_TRY(launch_psf_lobe(c->cT, c->psf_lobe, c->N, c->L, 4, st));
  // transfer functions: Hhat = FFT2(ifftshift(psf)), P = w |Hhat|^2 / N^2
  const float inv_n2 = 1.f / ((float)c->N * c->N);
  MF_TRY(launch_rows_r2c(c->cT, c->S, c->L, c->g, c->tw, true, st));
  MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, COL_FWD, nullptr, nullptr, 1.f, c->Hhat_T, st));
  MF_TRY(launch_power_spectrum(c->Hhat_T, c->P_T, c->chan_w, (long long)c->g.pitch * c->N, c->L, inv_n2, st));
  // b = w H^dagger y
  MF_TRY(launch_rows_r2c(c->Y, c->S, c->L, c->g, c->tw, false, st));
  MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, COL_CPLX_CONJ, nullptr, c->Hhat_T, inv_n2, nullptr, st));
  MF_TRY(launch_rows_c2r(c->S, c->L, c->g, c->tw, EPI_STORE, c->B, nullptr, nullptr, 0.f, nullptr, nullptr, nullptr,
                         nullptr, st));
  if (c->chan_w) MF_TRY(launch_scale_channels(c->B, c->chan_w, c->npix, c->L, st));
  // beta = max_l w_l max_k |H_l(k)|^2 and ||W_s||^2 (FP64)
  MF_TRY(launch_reduce_max(c->P_T, spec, (double)c->N * (double)c->N, c->partial, c->dres + 4, st));
  MF_TRY(launch_frame_bound(c->N, c->J, c->gen, c->omega_c, c->partial, c->dres + 5, st));
  double hs[16];
  MF_HIP(hipMemcpyAsync(hs, c->dres, sizeof(hs), hipMemcpyDeviceToHost, st));
  MF_HIP(hipStreamSynchronize(st));
  c->beta = hs[4];
  c->Ws2 = hs[5];
  c->K2 = p->mu_s * p->mu_s * c->Ws2 + p->mu_lambda * p->mu_lambda;
  c->tau = p->tau > 0 ? p->tau : 0.99 / (c->beta / 2.0 + c->sigma * c->K2);
  const double margin = 1.0 / c->tau - c->sigma * c->K2;
  if (!(margin > c->beta / 2.0))
    return set_error("step sizes violate 1/tau - sigma ||K||^2 > beta/2"), MUFFIN_ESTEP;
  c->delta = 2.0 - (c->beta / 2.0) / margin;
  if (!(c->rho < c->delta)) return set_error("rho must lie in (0, delta)"), MUFFIN_ESTEP;

  MF_HIP(hipMemsetAsync(c->X, 0, sizeof(float) * cube, st));
  MF_HIP(hipMemsetAsync(c->U, 0, sizeof(float) * cube * (c->J + 1), st));
  MF_HIP(hipMemsetAsync(c->V, 0, sizeof(float) * cube, st));
  MF_HIP(hipMemsetAsync(c->D, 0, sizeof(float) * cube, st));
  MF_HIP(hipStreamSynchronize(st));
  return MUFFIN_OK;
}

// Capture one iteration into a graph (capture records the work without running it).
int ensure_graph(muffin_ctx* c) {
  if (c->gexec) return MUFFIN_OK;
  MF_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_iteration(c, nullptr);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(c->st, &gr);
  if (rc != MUFFIN_OK) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  MF_HIP(e);
  c->graph = gr;
  MF_HIP(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  return MUFFIN_OK;
}

constexpr uint64_t kMagic = 0x4d5546464e434b31ull;  // "MUFFNCK1"
struct BlobHeader {
  uint64_t magic;
  int32_t N, L, J, gen, pc, pad;
  double mu_s, mu_l, tau, sigma, rho;
  int64_t iter;
};

}  // namespace

// ================================================================== C ABI
extern "C" {

const char* muffin_last_error(void) { return g_err.c_str(); }

const char* muffin_strerror(int code) {
  switch (code) {
    case MUFFIN_OK: return "ok";
    case MUFFIN_EINVAL: return "invalid argument";
    case MUFFIN_ENOMEM: return "out of memory";
    case MUFFIN_EHIP: return "HIP runtime error";
    case MUFFIN_ENONFINITE: return "non-finite value";
    case MUFFIN_ESTEP: return "step sizes violate the convergence condition";
    case MUFFIN_ESTATE: return "checkpoint does not match the context";
    default: return "unknown error";
  }
}

int muffin_init(muffin_ctx** out, const muffin_params* p, const float* dirty, const float* psf,
                int inputs_on_device, void* hip_stream) {
  if (!out) return set_error("out is NULL"), MUFFIN_EINVAL;
  *out = nullptr;
  MF_TRY(validate(p));
  if (!dirty || !psf) return set_error("dirty or psf is NULL"), MUFFIN_EINVAL;
  muffin_ctx* c = new (std::nothrow) muffin_ctx();
  if (!c) return set_error("host allocation failed"), MUFFIN_ENOMEM;
  c->user = (hipStream_t)hip_stream;
  const int rc = init_impl(c, p, dirty, psf, inputs_on_device);
  if (rc != MUFFIN_OK) {
    destroy(c);
    return rc;
  }
  *out = c;
  return MUFFIN_OK;
}

void muffin_free(muffin_ctx* c) { destroy(c); }

int muffin_step(muffin_ctx* c, int32_t n_iter) {
  if (!c || n_iter < 0) return set_error("bad context or n_iter"), MUFFIN_EINVAL;
  if (n_iter == 0) return MUFFIN_OK;
  StreamScope scope(c);
  if (!scope.ok) return set_error("stream ordering failed"), MUFFIN_EHIP;
  MF_TRY(ensure_graph(c));
  for (int i = 0; i < n_iter; ++i) MF_HIP(hipGraphLaunch(c->gexec, c->st));
  c->iter += n_iter;
  return MUFFIN_OK;
}

int muffin_step_timed(muffin_ctx* c, int32_t n_iter, double* ms) {
  if (!c || !ms || n_iter < 1) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  if (!scope.ok) return set_error("stream ordering failed"), MUFFIN_EHIP;
  MF_TRY(ensure_graph(c));
  MF_HIP(hipEventRecord(c->e0, c->st));
  for (int i = 0; i < n_iter; ++i) MF_HIP(hipGraphLaunch(c->gexec, c->st));
  MF_HIP(hipEventRecord(c->e1, c->st));
  MF_HIP(hipEventSynchronize(c->e1));
  float t = 0.f;
  MF_HIP(hipEventElapsedTime(&t, c->e0, c->e1));
  *ms = t;
  c->iter += n_iter;
  return MUFFIN_OK;
}

int muffin_profile(muffin_ctx* c, int32_t n_iter, double ms[8]) {
  if (!c || !ms || n_iter < 1) return set_error("bad arguments"), MUFFIN_EINVAL;
  for (int i = 0; i < 8; ++i) ms[i] = 0;
  StreamScope scope(c);
  int n_ad = 0, n_an = 0;
  for (int it = 0; it < n_iter; ++it) {
    // alternate which kernel family is bracketed so the marks do not pile up in one iteration
    const int fam = 1 + (it & 1);
    MF_TRY(enqueue_iteration(c, c->ph, c->gen == 2 ? fam : 0));
    MF_HIP(hipEventSynchronize(c->ph[4]));
    float t[4];
    for (int k = 0; k < 4; ++k) MF_HIP(hipEventElapsedTime(&t[k], c->ph[k], c->ph[k + 1]));
    for (int k = 0; k < 4; ++k) {
      ms[k + 1] += t[k] / n_iter;
      ms[0] += t[k] / n_iter;
    }
    if (c->gen == 2) {
      for (int j = 0; j < c->J; ++j) {
        if (!atrous_double_fits(c->N, j, nullptr, nullptr)) continue;
        float tk = 0.f;
        MF_HIP(hipEventElapsedTime(&tk, c->kev[2 * j], c->kev[2 * j + 1]));
        if (fam == 1) {
          ms[6] += tk;
          ++n_ad;
        } else {
          ms[5] += tk;
          ++n_an;
        }
      }
    }
  }
  if (n_an) ms[5] /= n_an;
  if (n_ad) ms[6] /= n_ad;
  c->iter += n_iter;
  return MUFFIN_OK;
}

int muffin_objective(muffin_ctx* c, double out[4]) {
  if (!c || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  MF_TRY(enqueue_objective(c));
  double h[4];
  MF_HIP(hipMemcpyAsync(h, c->dres, sizeof(h), hipMemcpyDeviceToHost, c->st));
  MF_HIP(hipStreamSynchronize(c->st));
  out[1] = h[1];
  out[2] = c->p.mu_s * h[2];
  out[3] = c->p.mu_lambda * h[3];
  out[0] = out[1] + out[2] + out[3];
  if (!std::isfinite(out[0])) return set_error("objective is not finite"), MUFFIN_ENONFINITE;
  return MUFFIN_OK;
}

int muffin_solve(muffin_ctx* c, int32_t max_iter, int32_t check_every, double tol, double f_ref,
                 int32_t* iters_done, double* f_final) {
  if (!c || max_iter < 0 || check_every < 1 || !(tol >= 0)) return set_error("bad arguments"), MUFFIN_EINVAL;
  int done = 0;
  double f = NAN, f_prev = NAN, o[4];
  while (done < max_iter) {
    const int n = (max_iter - done < check_every) ? max_iter - done : check_every;
    MF_TRY(muffin_step(c, n));
    done += n;
    const int rc = muffin_objective(c, o);
    f = o[0];
    if (rc != MUFFIN_OK) {
      if (iters_done) *iters_done = done;
      if (f_final) *f_final = f;
      return rc;
    }
    if (std::isfinite(f_ref)) {
      if ((f - f_ref) / std::fabs(f_ref) <= tol) break;
    } else if (std::isfinite(f_prev) && std::fabs(f - f_prev) <= tol * std::fabs(f)) {
      break;
    }
    f_prev = f;
  }
  if (iters_done) *iters_done = done;
  if (f_final) *f_final = f;
  return MUFFIN_OK;
}

int muffin_info(muffin_ctx* c, double out[8]) {
  if (!c || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  out[0] = c->tau;
  out[1] = c->sigma;
  out[2] = c->rho;
  out[3] = c->beta;
  out[4] = c->K2;
  out[5] = c->Ws2;
  out[6] = c->delta;
  out[7] = (double)c->iter;
  return MUFFIN_OK;
}

int muffin_set_x(muffin_ctx* c, const float* x0, int on_device) {
  if (!c || !x0) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  MF_TRY(copy_in(c->X, x0, c->cube, on_device, c->st));
  MF_TRY(launch_clamp_pos(c->X, c->cube, c->st));
  MF_HIP(hipMemsetAsync(c->U, 0, sizeof(float) * c->cube * (c->J + 1), c->st));
  MF_HIP(hipMemsetAsync(c->V, 0, sizeof(float) * c->cube, c->st));
  return MUFFIN_OK;
}

int muffin_get_x(muffin_ctx* c, float* x, int on_device) {
  if (!c || !x) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  return copy_out(x, c->X, c->cube, on_device, c->st);
}
int muffin_get_u(muffin_ctx* c, float* u, int on_device) {
  if (!c || !u) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  return copy_out(u, c->U, c->cube * (c->J + 1), on_device, c->st);
}
int muffin_get_v(muffin_ctx* c, float* v, int on_device) {
  if (!c || !v) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  return copy_out(v, c->V, c->cube, on_device, c->st);
}

int muffin_state_size(muffin_ctx* c, size_t* bytes) {
  if (!c || !bytes) return set_error("bad arguments"), MUFFIN_EINVAL;
  *bytes = sizeof(BlobHeader) + sizeof(float) * (size_t)c->cube * (c->J + 3);
  return MUFFIN_OK;
}

int muffin_get_state(muffin_ctx* c, void* blob, size_t bytes) {
  size_t need = 0;
  MF_TRY(muffin_state_size(c, &need));
  if (!blob || bytes < need) return set_error("blob too small"), MUFFIN_EINVAL;
  BlobHeader h{};
  h.magic = kMagic;
  h.N = c->N;
  h.L = c->L;
  h.J = c->J;
  h.gen = c->gen;
  h.pc = c->p.penalize_coarse;
  h.mu_s = c->p.mu_s;
  h.mu_l = c->p.mu_lambda;
  h.tau = c->tau;
  h.sigma = c->sigma;
  h.rho = c->rho;
  h.iter = c->iter;
  std::memcpy(blob, &h, sizeof(h));
  float* f = (float*)((char*)blob + sizeof(h));
  StreamScope scope(c);
  MF_TRY(copy_out(f, c->X, c->cube, 0, c->st));
  MF_TRY(copy_out(f + c->cube, c->U, c->cube * (c->J + 1), 0, c->st));
  MF_TRY(copy_out(f + c->cube * (c->J + 2), c->V, c->cube, 0, c->st));
  return MUFFIN_OK;
}

int muffin_set_state(muffin_ctx* c, const void* blob, size_t bytes) {
  size_t need = 0;
  MF_TRY(muffin_state_size(c, &need));
  if (!blob || bytes < need) return set_error("blob too small"), MUFFIN_ESTATE;
  BlobHeader h;
  std::memcpy(&h, blob, sizeof(h));
  if (h.magic != kMagic || h.N != c->N || h.L != c->L || h.J != c->J || h.gen != c->gen ||
      h.pc != c->p.penalize_coarse || h.mu_s != c->p.mu_s || h.mu_l != c->p.mu_lambda || h.tau != c->tau ||
      h.sigma != c->sigma || h.rho != c->rho)
    return set_error("checkpoint sizes or parameters differ from the context"), MUFFIN_ESTATE;
  const float* f = (const float*)((const char*)blob + sizeof(h));
  StreamScope scope(c);
  MF_TRY(copy_in(c->X, f, c->cube, 0, c->st));
  MF_TRY(copy_in(c->U, f + c->cube, c->cube * (c->J + 1), 0, c->st));
  MF_TRY(copy_in(c->V, f + c->cube * (c->J + 2), c->cube, 0, c->st));
  c->iter = h.iter;
  return MUFFIN_OK;
}

int muffin_warm_start(muffin_ctx* c, muffin_cnn* net) {
  if (!c || !net) return set_error("bad arguments"), MUFFIN_EINVAL;
  if (c->N % 32) return set_error("warm start needs N to be a multiple of 32"), MUFFIN_EINVAL;
  StreamScope scope(c);
  MF_TRY(cnn_warm_input(c->Y, c->psf_lobe, c->cA, c->N, c->L, c->st));
  MF_HIP(hipStreamSynchronize(c->st));
  MF_TRY(muffin_cnn_predict(net, c->cA, c->cB, c->L, c->N));
  MF_HIP(hipDeviceSynchronize());
  MF_HIP(hipMemcpyAsync(c->X, c->cB, sizeof(float) * c->cube, hipMemcpyDeviceToDevice, c->st));
  MF_TRY(launch_clamp_pos(c->X, c->cube, c->st));
  MF_HIP(hipMemsetAsync(c->U, 0, sizeof(float) * c->cube * (c->J + 1), c->st));
  MF_HIP(hipMemsetAsync(c->V, 0, sizeof(float) * c->cube, c->st));
  return MUFFIN_OK;
}

int muffin_apply_op(muffin_ctx* c, int op, const float* in, float* out) {
  if (!c || !in || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  const long long np = c->npix;
  const float inv_n2 = 1.f / ((float)c->N * c->N);
  switch (op) {
    case MUFFIN_OP_H:
    case MUFFIN_OP_HT:
      MF_TRY(launch_rows_r2c(in, c->S, c->L, c->g, c->tw, false, c->st));
      MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, op == MUFFIN_OP_H ? COL_CPLX : COL_CPLX_CONJ, nullptr, c->Hhat_T,
                         inv_n2, nullptr, c->st));
      MF_TRY(launch_rows_c2r(c->S, c->L, c->g, c->tw, EPI_STORE, out, nullptr, nullptr, 0.f, nullptr, nullptr,
                             nullptr, nullptr, c->st));
      return MUFFIN_OK;
    case MUFFIN_OP_GRAD:
      return enqueue_gradient(c, in, out, nullptr, 0.f);
    case MUFFIN_OP_IUWT: {
      const long long ucs = (long long)(c->J + 1) * np;
      const float* cur = in;
      float* bufs[2] = {c->cA, c->cB};
      for (int j = 0; j < c->J; ++j) {
        float* nxt = bufs[j & 1];
        MF_TRY(launch_atrous(SM_SMOOTH, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(nxt, np),
                             PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
        float* wj = out + (long long)j * np;
        if (c->gen == 2) {
          // w = c_j - H_j c_{j+1}: smooth c_{j+1} into the output plane, then subtract
          MF_TRY(launch_atrous(SM_SMOOTH, c->N, c->L, j, pref(nxt, np), PlaneRef{}, PlaneRef{}, pout(c->cT, np),
                               PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
          MF_TRY(launch_pointwise(PT_SUB, c->N, c->L, pref(c->cT, np), pref(cur, np), pout(wj, ucs), 0.f, 1.f,
                                  nullptr, nullptr, c->st));
        } else {
          MF_TRY(launch_pointwise(PT_SUB, c->N, c->L, pref(nxt, np), pref(cur, np), pout(wj, ucs), 0.f, 1.f, nullptr,
                                  nullptr, c->st));
        }
        cur = nxt;
      }
      return launch_pointwise(PT_COPY, c->N, c->L, pref(cur, np), PlaneRef{},
                              pout(out + (long long)c->J * np, ucs), 1.f, 1.f, nullptr, nullptr, c->st);
    }
    case MUFFIN_OP_IUWT_ADJ: {
      const float* a = nullptr;
      MF_TRY(enqueue_adjoint(c, in, (long long)(c->J + 1) * np, 1.f, &a));
      return launch_pointwise(PT_COPY, c->N, c->L, pref(a, np), PlaneRef{}, pout(out, np), 1.f, 1.f, nullptr,
                              nullptr, c->st);
    }
    case MUFFIN_OP_DCT:
      return launch_dct(in, out, c->WT, np, c->L, c->st);
    case MUFFIN_OP_IDCT:
      return launch_dct(in, out, c->W, np, c->L, c->st);
    default:
      return set_error("unknown operator"), MUFFIN_EINVAL;
  }
}

}  // extern "C"
