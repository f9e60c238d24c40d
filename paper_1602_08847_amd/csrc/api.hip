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

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
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
int launch_scale_channels(float* x, const float* chan_w, long long npix, long long cs, int nch, hipStream_t st);
int cnn_warm_input(const float* Y, long long cs, const float* scale, float* out, int N, int L, hipStream_t st);
int cnn_predict_after(muffin_cnn* net, const float* in, float* out, int B, int N, hipStream_t after);
int launch_psf_lobe(const float* psf, long long cs, float* out, int N, int L, int radius, hipStream_t st);
}  // namespace mf

using namespace mf;

// One cube of a context: its channels [ch0, ch0 + L) of the packed arrays, its spectral weight and
// step sizes, and its cosine-transform tables.  A context built by muffin_init holds one segment;
// a batch group holds every cube of one image side.
struct Seg {
  int ch0 = 0, L = 0;
  double mu_l = 0, tau = 0, beta = 0, K2 = 0, delta = 0;
  float *W = nullptr, *WT = nullptr;
  float2 *twL = nullptr, *csL = nullptr;
  float2* blu = nullptr;  // Bluestein table when L has no FFT plan (spectral_blu_table)
};

struct muffin_ctx {
  muffin_params p{};
  std::vector<Seg> segs;
  std::vector<float> chan_w_host;
  int N = 0, L = 0, J = 0, gen = 2;
  // spatial prior: the IUWT (np_u = J + 1 dual planes per channel) or the union of Daubechies
  // bases (np_u = kUobBases planes, each one basis's pyramid of coefficients)
  bool uob = false;
  int np_u = 0;
  UobFilters uf{};
  float *uobA = nullptr, *uobB = nullptr;  // approximations between levels: (N/2)^2 and (N/4)^2 per (channel, basis)
  // Every N x N plane of the cube buffers sits in a slot of cs floats: N^2 plus one row, rounded up
  // to 32 floats, plus 32 more (128 bytes).  The spectral step walks each pixel across all the
  // channels; with planes a power of two apart those accesses fall on few HBM channels, and the
  // extra 128 bytes spread them (at 1024^2 x 256 the step runs 1.8 -> 1.4 ms, while the row-wise
  // IUWT kernels keep their speed).  cube = cs * L.  The planes of U, which are only walked row by
  // row, are us floats apart (ucube = us * L * (J + 1)).
  long long npix = 0, cs = 0, cube = 0, us = 0, ucube = 0;
  FftGeom g;
  int device = 0;
  hipStream_t user = nullptr, st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, e0 = nullptr, e1 = nullptr;
  hipEvent_t ph[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t kev[16] = {};  // per-launch timing marks of one kernel family (profiling only)
  int kkind[8] = {};        // launch kind of each bracketed launch
  int nk = 0;               // bracketed launches
  float *X = nullptr, *U = nullptr, *V = nullptr, *D = nullptr, *Q = nullptr, *B = nullptr, *Y = nullptr;
  float *cA = nullptr, *cB = nullptr, *cT = nullptr;
  float2* S = nullptr;
  float2* Hhat_T = nullptr;
  float* P_T = nullptr;
  float2* tw = nullptr;
  float* chan_w = nullptr;
  float* psf_lobe = nullptr;  // [L] sum of each PSF over the 9 x 9 window at its origin
  double* partial = nullptr;
  double* dres = nullptr;  // device scalars: [1..3] objective terms, [5] ||W_s||^2, [6..11] convergence
                           // norms, [12..13] SNR sums
  // Every cube of the context has mu_lambda = 0 (the paper's first calibration step, Sec. 4): the
  // spectral term of the primal step vanishes, so the primal step runs in the gradient's last pass
  // channel by channel (with each channel's tau from tau_ch) and the spectral kernel is skipped; V
  // then never changes (it stays saturated, and sat(V) = V).
  bool local_primal = false;
  float* tau_ch = nullptr;  // [L] tau of each channel's cube (FP32, as the spectral kernel uses it)
  // copies of X, U (dense [L][J+1] planes) and V before a monitored iteration (allocated on first use)
  float *Xs = nullptr, *Us = nullptr, *Vs = nullptr;
  double sigma = 1, rho = 1, Ws2 = 0;
  float omega_c = 1.f;
  long long iter = 0;
  // Fused tail (second generation, coarse plane penalised, last group a pair: fused_ok; whether
  // it runs: fused, see MUFFIN_FLAG_FUSED_TAIL): the last analysis
  // launch also runs the next iteration's first adjoint pair on the planes it has just updated
  // (PR_FUSED).  Those three planes (scales jf, jf + 1 and the coarse plane) alternate between U
  // and U2 ([L][3] planes, us floats apart) from one iteration to the next, so that a band's halo
  // still reads the old values; upar names the buffer holding the current ones (0: U, 1: U2).
  // Acar carries the adjoint's running sum after that pair into the next iteration; acar_ok is
  // false when U was set from outside and Acar has to be recomputed.
  bool fused_ok = false, fused = false, acar_ok = true;
  int jf = 0, upar = 0;
  float *U2 = nullptr, *Acar = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};  // one iteration per parity of upar
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // Visibility-domain data term (Sec. 2, eq. (viseq)) in place of H: K visibilities per channel,
  // each with its baseline in wavelengths of the channel and the residual the forward pass leaves
  // (vp, [L][K]); the data (vdata, [L][K] complex); the forward pass's band sums (vpart,
  // [vC][L][K]); l = m of each column or row (vlt, FP64 [N]); n (vnt, FP64 [N][N]) and 1/n
  // (vinvn, FP32) of each pixel; x / n of the cube (XN, dense [L][N][N]); the staging buffer of
  // muffin_vis_residual for host output (vres, [L][K] complex, allocated on its first such call).
  // The image-plane buffers (Y, B, S, Hhat_T, P_T, psf_lobe) are then not allocated.
  bool vis = false;
  int K = 0, vC = 0;
  VisPt* vp = nullptr;
  float2 *vdata = nullptr, *vpart = nullptr, *vres = nullptr;
  double *vlt = nullptr, *vnt = nullptr;
  float *vinvn = nullptr, *XN = nullptr;
};

// Visibility inputs of muffin_init_vis.
struct VisInit {
  const muffin_vis_desc* d;
  const float* vis;
  int on_device;
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
  if (p->flags & ~(MUFFIN_FLAG_SINGLE_SCALE | MUFFIN_FLAG_NO_FUSED_TAIL | MUFFIN_FLAG_FUSED_TAIL |
                   MUFFIN_FLAG_UOB_ALL_BASES | MUFFIN_FLAG_UOB_PER_BASIS | MUFFIN_FLAG_SPECTRAL_DENSE |
                   MUFFIN_FLAG_SPECTRAL_BLUESTEIN))
    return set_error("unknown flags"), MUFFIN_EINVAL;
  if ((p->flags & MUFFIN_FLAG_NO_FUSED_TAIL) && (p->flags & MUFFIN_FLAG_FUSED_TAIL))
    return set_error("FUSED_TAIL and NO_FUSED_TAIL exclude each other"), MUFFIN_EINVAL;
  if ((p->flags & MUFFIN_FLAG_UOB_ALL_BASES) && (p->flags & MUFFIN_FLAG_UOB_PER_BASIS))
    return set_error("UOB_ALL_BASES and UOB_PER_BASIS exclude each other"), MUFFIN_EINVAL;
  if ((p->flags & MUFFIN_FLAG_SPECTRAL_DENSE) && (p->flags & MUFFIN_FLAG_SPECTRAL_BLUESTEIN))
    return set_error("SPECTRAL_DENSE and SPECTRAL_BLUESTEIN exclude each other"), MUFFIN_EINVAL;
  if (p->iuwt_gen != 1 && p->iuwt_gen != 2) return set_error("iuwt_gen must be 1 or 2"), MUFFIN_EINVAL;
  if (p->prior != MUFFIN_PRIOR_IUWT && p->prior != MUFFIN_PRIOR_UOB)
    return set_error("prior must be MUFFIN_PRIOR_IUWT or MUFFIN_PRIOR_UOB"), MUFFIN_EINVAL;
  if (p->prior == MUFFIN_PRIOR_UOB && p->N % (1 << p->J) != 0)
    return set_error("the union of bases needs N divisible by 2^J"), MUFFIN_EINVAL;
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
// Launch kinds reported by muffin_profile.
enum LaunchKind { K_DB_ANALYSIS = 0, K_DB_ADJOINT = 1, K_DB_ANALYSIS_C = 2, K_PR_ANALYSIS = 3, K_PR_ADJOINT = 4,
                  K_PR_ANALYSIS_C = 5, K_TR_ANALYSIS = 6, K_TR_ADJOINT = 7, K_TR_ANALYSIS_C = 8, K_PR_FUSED = 9, K_KINDS = 12 };

// Brackets one launch with timing marks when timed (at most 8 per family).
template <class F>
static int timed_launch(muffin_ctx* c, bool timed, int kind, F&& launch) {
  timed = timed && c->nk < 8;
  if (timed) MF_HIP(hipEventRecord(c->kev[2 * c->nk], c->st));
  MF_TRY(launch());
  if (timed) {
    MF_HIP(hipEventRecord(c->kev[2 * c->nk + 1], c->st));
    c->kkind[c->nk++] = kind;
  }
  return MUFFIN_OK;
}

static bool use_pairs(const muffin_ctx* c) { return c->gen == 2 && !(c->p.flags & MUFFIN_FLAG_SINGLE_SCALE); }

// Plane k of U in the buffers of parity par (see muffin_ctx::upar): pointer and channel stride.
static PlaneOut uplane(const muffin_ctx* c, int k, int par) {
  if (c->fused && par && k >= c->jf) return PlaneOut{c->U2 + (long long)(k - c->jf) * c->us, 3 * c->us};
  return PlaneOut{c->U + (long long)k * c->us, (long long)c->np_u * c->us};
}
static PlaneRef uref(const muffin_ctx* c, int k, int par) {
  const PlaneOut o = uplane(c, k, par);
  return PlaneRef{o.p, o.cs};
}

// The band, pair and triple launches of the two IUWT phases, in order; j is the finest scale of a
// launch.  Consecutive scales are grouped into one launch each, from the finest scale up: J = 1..6
// gives groups of 1; 2; 3; 2, 2; 3, 2; 3, 3 scales (at J = 4 two pairs move as few bytes as a
// triple and a single scale, with smaller halos).  The adjoint runs the same groups from the
// coarsest scale down.
struct IuwtStep {
  int mode, j;
  const char* name;
};

static std::vector<int> iuwt_groups(const muffin_ctx* c) {
  const int J = c->J;
  if (c->p.flags & MUFFIN_FLAG_SINGLE_SCALE) return std::vector<int>(J, 1);
  // first generation: pairs only, a single scale first so that the last analysis group is a pair
  // and takes the coarse plane's dual step
  static const std::vector<int> g1[7] = {{}, {1}, {2}, {1, 2}, {2, 2}, {1, 2, 2}, {2, 2, 2}};
  static const std::vector<int> g[7] = {{}, {1}, {2}, {3}, {2, 2}, {3, 2}, {3, 3}};
  return c->gen == 1 ? g1[J] : g[J];
}

static std::vector<IuwtStep> analysis_schedule(const muffin_ctx* c) {
  const bool coarse = c->omega_c != 0.f;
  const std::vector<int> groups = iuwt_groups(c);
  std::vector<IuwtStep> v;
  int j = 0;
  for (size_t k = 0; k < groups.size(); ++k) {
    const bool last = k + 1 == groups.size() && coarse;
    switch (groups[k]) {
      case 3: v.push_back({last ? TR_ANALYSIS_C : TR_ANALYSIS, j, "analysis triple"}); break;
      case 2:
        if (c->gen == 1) v.push_back({last ? P1_ANALYSIS_C : P1_ANALYSIS, j, "analysis pair"});
        else if (last && c->fused) v.push_back({PR_FUSED, j, "analysis pair + next adjoint pair"});
        else v.push_back({last ? PR_ANALYSIS_C : PR_ANALYSIS, j, "analysis pair"});
        break;
      default:
        if (c->gen == 1) v.push_back({SM_DETAIL1, j, "analysis"});
        else v.push_back({last ? DB_ANALYSIS_C : DB_ANALYSIS, j, "analysis"});
    }
    j += groups[k];
  }
  return v;
}

static std::vector<IuwtStep> adjoint_schedule(const muffin_ctx* c) {
  const std::vector<int> groups = iuwt_groups(c);
  std::vector<IuwtStep> v;
  int top = c->J;  // one past the coarsest scale left
  for (size_t k = groups.size(); k-- > 0;) {
    const int j = top - groups[k];
    switch (groups[k]) {
      case 3: v.push_back({TR_ADJOINT, j, "adjoint triple"}); break;
      case 2: v.push_back({c->gen == 1 ? P1_ADJOINT : PR_ADJOINT, j, "adjoint pair"}); break;
      default: v.push_back({c->gen == 1 ? SM_SUBADD : DB_ADJOINT, j, "adjoint"});
    }
    top = j;
  }
  return v;
}

// ---------------------------------------------------------------- union of bases
// Approximation planes between levels: LL_l of every (channel, basis) sits in uobA when l is odd
// ((N/2)^2 floats each) and in uobB when l is even ((N/4)^2 floats each).
static long long uob_cap(const muffin_ctx* c, int level) {
  const long long h = c->N >> ((level & 1) ? 1 : 2);
  return h * h > 0 ? h * h : 1;
}
static float* uob_ll(const muffin_ctx* c, int level, int ch0) {
  return ((level & 1) ? c->uobA : c->uobB) + (long long)ch0 * kUobBases * uob_cap(c, level);
}

// Workgroup layout of the union-of-bases levels after the first (flags; -1: by the level's size).
static int uob_all_bases(const muffin_ctx* c) {
  if (c->p.flags & MUFFIN_FLAG_UOB_ALL_BASES) return 1;
  if (c->p.flags & MUFFIN_FLAG_UOB_PER_BASIS) return 0;
  return -1;
}

// W_s of nch channel images (in, channel stride in_cs; channel ch0 of the context) through the J
// levels of every basis: UOB_DUAL updates the dual planes U (strides u_cs, u_bs) with
// u <- rho sat(u + coef w) + (1 - rho) u, UOB_STORE writes scale * w to out, UOB_ABS adds
// sum |scale * w| (FP64) to *dst_abs.
int enqueue_uob_analysis(muffin_ctx* c, int mode, const float* in, long long in_cs, int ch0, int nch, float* U,
                         long long u_cs, long long u_bs, float* out, long long out_cs, long long out_bs, float coef,
                         float rho, float scale, double* dst_abs) {
  for (int lev = 1; lev <= c->J; ++lev) {
    UobLevelArgs a;
    a.f = c->uf;
    a.all_bases = uob_all_bases(c);
    a.n = c->N >> (lev - 1);
    a.N = c->N;
    if (lev == 1) {
      a.in = in;
      a.in_cs = in_cs;
      a.in_bs = 0;
      a.in_ld = c->N;
      a.shared_input = 1;
    } else {
      a.in = uob_ll(c, lev - 1, ch0);
      a.in_cs = kUobBases * uob_cap(c, lev - 1);
      a.in_bs = uob_cap(c, lev - 1);
      a.in_ld = a.n;
    }
    a.last = lev == c->J;
    if (!a.last) {
      a.llout = uob_ll(c, lev, ch0);
      a.ll_cs = kUobBases * uob_cap(c, lev);
      a.ll_bs = uob_cap(c, lev);
    }
    a.U = U;
    a.u_cs = u_cs;
    a.u_bs = u_bs;
    a.out = out;
    a.out_cs = out_cs;
    a.out_bs = out_bs;
    a.coef = coef;
    a.rho = rho;
    a.scale = scale;
    int nb = 0;
    MF_TRY(launch_uob_an(mode, a, nch, c->partial, &nb, c->st));
    if (mode == UOB_ABS) MF_TRY(launch_reduce_sum(c->partial, nb, dst_abs, 1, c->st));
  }
  return MUFFIN_OK;
}

// dst = W_s^dagger u = sum_n Psi_n^T u_n / sqrt(8) for every channel (dst channel stride dst_cs).
int enqueue_uob_adjoint(muffin_ctx* c, const float* U, long long u_cs, long long u_bs, float* dst, long long dst_cs) {
  for (int lev = c->J; lev >= 1; --lev) {
    UobLevelArgs a;
    a.f = c->uf;
    a.all_bases = uob_all_bases(c);
    a.n = c->N >> (lev - 1);
    a.N = c->N;
    if (lev == c->J) {
      a.in = U;
      a.in_cs = u_cs;
      a.in_bs = u_bs;
      a.in_ld = c->N;
    } else {
      a.in = uob_ll(c, lev, 0);
      a.in_cs = kUobBases * uob_cap(c, lev);
      a.in_bs = uob_cap(c, lev);
      a.in_ld = c->N >> lev;
    }
    a.U = const_cast<float*>(U);
    a.u_cs = u_cs;
    a.u_bs = u_bs;
    if (lev == 1) {
      a.out = dst;
      a.out_cs = dst_cs;
      a.scale = (float)(1.0 / std::sqrt((double)kUobBases));
      MF_TRY(launch_uob_adj(true, a, c->L, c->st));
    } else {
      a.llout = uob_ll(c, lev - 1, 0);
      a.ll_cs = kUobBases * uob_cap(c, lev - 1);
      a.ll_bs = uob_cap(c, lev - 1);
      MF_TRY(launch_uob_adj(false, a, c->L, c->st));
    }
  }
  return MUFFIN_OK;
}

// Spatial adjoint of omega-weighted U; returns the buffer holding a = W_s^dagger (omega u).
// Second generation: Horner steps a <- u_j + H_j (a - H_j u_j) from the coarsest scale down, two
// scales per launch where possible.
// Ubase: plane j of channel l at Ubase + l ucs + j ups.  The result has channel stride cs.  With
// carried, the first launch of the schedule is skipped and the Horner steps start from that plane
// (channel stride cs): the fused tail of the last iteration has already run them.
int enqueue_adjoint(muffin_ctx* c, const float* Ubase, long long ups, long long ucs, float omega_c,
                    const float** result, bool timed = false, const float* carried = nullptr) {
  if (c->uob) {
    MF_TRY(enqueue_uob_adjoint(c, Ubase, ucs, ups, c->cA, c->cs));
    *result = c->cA;
    return MUFFIN_OK;
  }
  const int J = c->J;
  const long long np = c->cs;
  const float* a = Ubase + (long long)J * ups;  // coarse plane
  long long acs = ucs;
  float* bufs[2] = {c->cA, c->cB};
  int nb = 0;
  std::vector<IuwtStep> sched = adjoint_schedule(c);
  if (carried) {
    sched.erase(sched.begin());
    a = carried;
    acs = np;
  } else if (omega_c != 1.f) {
    MF_TRY(launch_pointwise(PT_COPY, c->N, c->L, pref(a, acs), PlaneRef{}, pout(c->cA, np), omega_c, 1.f, nullptr,
                            nullptr, c->st));
    a = c->cA;
    acs = np;
    nb = 1;
  }
  for (const IuwtStep& st : sched) {
    float* dst = bufs[nb];
    const int j = st.j;
    const float* uj = Ubase + (long long)j * ups;
    if (st.mode == TR_ADJOINT) {
      // steps j + 2, j + 1, j
      MF_TRY(timed_launch(c, timed, K_TR_ADJOINT, [&] {
        return launch_triple(TR_ADJOINT, c->N, c->L, j, pref(Ubase + (long long)(j + 2) * ups, ucs),
                             pref(Ubase + (long long)(j + 1) * ups, ucs), pref(uj, ucs), pref(a, acs), pout(dst, np),
                             PlaneOut{}, PlaneOut{}, PlaneOut{}, 0.f, 1.f, 0.f, c->st);
      }));
    } else if (st.mode == PR_ADJOINT || st.mode == P1_ADJOINT) {
      // steps j + 1 then j
      const float* uh = Ubase + (long long)(j + 1) * ups;
      MF_TRY(timed_launch(c, timed, K_PR_ADJOINT, [&] {
        return launch_pair(st.mode, c->N, c->L, j, pref(uh, ucs), pref(uj, ucs), pref(a, acs), pout(dst, np),
                           PlaneOut{}, PlaneOut{}, 0.f, 1.f, 0.f, c->st);
      }));
    } else if (st.mode == DB_ADJOINT) {
      MF_TRY(timed_launch(c, timed, K_DB_ADJOINT, [&] {
        return launch_atrous(DB_ADJOINT, c->N, c->L, j, pref(uj, ucs), pref(a, acs), PlaneRef{}, pout(dst, np),
                             PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st);
      }));
    } else {
      MF_TRY(launch_atrous(SM_SUBADD, c->N, c->L, j, pref(a, acs), pref(uj, ucs), pref(uj, ucs), pout(dst, np),
                           PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
    }
    a = dst;
    acs = np;
    nb ^= 1;
  }
  *result = a;
  return MUFFIN_OK;
}

// Analysis of the channel images in (stride cs) fused with the spatial dual step on U; second
// generation: two scales per launch where possible, the last one feeding the coarse plane's step.
int enqueue_dual_update(muffin_ctx* c, const float* in, bool timed = false, int par = 0) {
  if (c->uob)
    return enqueue_uob_analysis(c, UOB_DUAL, in, c->cs, 0, c->L, c->U, (long long)c->np_u * c->us, c->us, nullptr, 0,
                                0, (float)(c->sigma * c->p.mu_s / std::sqrt((double)kUobBases)), (float)c->rho, 1.f,
                                nullptr);
  const int J = c->J;
  const long long np = c->cs, us = c->us, ucs = (long long)c->np_u * us;
  const float coef = (float)(c->sigma * c->p.mu_s);
  const float rho = (float)c->rho;
  const float coefc = coef * c->omega_c;
  const bool coarse = c->omega_c != 0.f;  // with omega = 0 on the coarse plane its dual stays put
  float* Uc = c->U + (long long)J * us;
  const float* cur = in;
  float* bufs[2] = {c->cA, c->cB};
  int nb = 0;
  for (const IuwtStep& st : analysis_schedule(c)) {
    float* nxt = bufs[nb];
    const int j = st.j;
    float* uj = c->U + (long long)j * us;
    switch (st.mode) {
      case PR_FUSED:
        MF_TRY(timed_launch(c, timed, K_PR_FUSED, [&] {
          return launch_fused_pair(c->N, c->L, j, pref(cur, np), uref(c, j, par), uref(c, j + 1, par),
                                   uref(c, J, par), uplane(c, j, par ^ 1), uplane(c, j + 1, par ^ 1),
                                   uplane(c, J, par ^ 1), pout(c->Acar, np), coef, rho, coefc, c->st);
        }));
        break;
      case SM_DETAIL1:
        MF_TRY(launch_atrous(SM_DETAIL1, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(uj, ucs),
                             pout(nxt, np), coef, rho, nullptr, nullptr, c->st));
        break;
      case P1_ANALYSIS_C:
      case P1_ANALYSIS:
      case PR_ANALYSIS_C:
      case PR_ANALYSIS: {
        float* uj1 = c->U + (long long)(j + 1) * us;
        const bool co = st.mode == PR_ANALYSIS_C || st.mode == P1_ANALYSIS_C;
        MF_TRY(timed_launch(c, timed, co ? K_PR_ANALYSIS_C : K_PR_ANALYSIS, [&] {
          return launch_pair(st.mode, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(uj, ucs),
                             pout(uj1, ucs), co ? pout(Uc, ucs) : pout(nxt, np), coef, rho, co ? coefc : 0.f, c->st);
        }));
        break;
      }
      case TR_ANALYSIS_C:
      case TR_ANALYSIS: {
        float* uj1 = c->U + (long long)(j + 1) * us;
        float* uj2 = c->U + (long long)(j + 2) * us;
        const bool co = st.mode == TR_ANALYSIS_C;
        MF_TRY(timed_launch(c, timed, co ? K_TR_ANALYSIS_C : K_TR_ANALYSIS, [&] {
          return launch_triple(st.mode, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, PlaneRef{},
                               pout(uj, ucs), pout(uj1, ucs), pout(uj2, ucs), co ? pout(Uc, ucs) : pout(nxt, np), coef,
                               rho, co ? coefc : 0.f, c->st);
        }));
        break;
      }
      case DB_ANALYSIS_C:
        MF_TRY(timed_launch(c, timed, K_DB_ANALYSIS_C, [&] {
          return launch_atrous(DB_ANALYSIS_C, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(uj, ucs),
                               pout(Uc, ucs), coef, rho, nullptr, nullptr, c->st, 0, coefc);
        }));
        break;
      default:
        MF_TRY(timed_launch(c, timed, K_DB_ANALYSIS, [&] {
          return launch_atrous(DB_ANALYSIS, c->N, c->L, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(uj, ucs),
                               pout(nxt, np), coef, rho, nullptr, nullptr, c->st);
        }));
    }
    cur = nxt;
    nb ^= 1;
  }
  // a first-generation schedule that ends with a single scale updates the coarse plane's dual here
  if (c->gen == 1 && coarse && analysis_schedule(c).back().mode == SM_DETAIL1)
    MF_TRY(launch_pointwise(PT_COARSE, c->N, c->L, pref(cur, np), PlaneRef{}, pout(Uc, ucs), coefc, rho, nullptr,
                            nullptr, c->st));
  return MUFFIN_OK;
}

// Phi_l (x_l) (x in slots of cs floats) into the band sums, then the residual r = Phi x + vsign vis
// (vis NULL: Phi x): w_l r into c->vp for the adjoint (weighted: the channel weights of eq. (reg),
// else 1), r itself into rout unless NULL, and 1/2 w_l |r|^2 block sums in partial unless NULL.
int enqueue_vis_forward(muffin_ctx* c, const float* x, long long xcs, const float2* vis, float vsign, double* partial,
                        int* nb, float2* rout = nullptr, bool weighted = true) {
  MF_TRY(launch_vis_xn(x, xcs, c->vinvn, c->XN, c->N, c->L, c->st));
  MF_TRY(launch_vis_fwd(c->vp, c->XN, c->vlt, c->vnt, c->vpart, c->N, c->K, c->L, c->vC, c->st));
  return launch_vis_resid(c->vpart, c->vC, c->L, c->K, vis, vsign, weighted ? c->chan_w : nullptr, c->vp, partial,
                          nb, rout, c->st);
}

int enqueue_gradient(muffin_ctx* c, const float* x, float* out, const float* s, float s_scale) {
  if (c->vis) {
    // Re Phi^H (Phi x - v) + s_scale s
    MF_TRY(enqueue_vis_forward(c, x, c->cs, c->vdata, -1.f, nullptr, nullptr));
    return launch_vis_adj(c->vp, c->K, c->L, c->vlt, c->vnt, c->vinvn, c->N, out, c->cs, s, c->cs, s_scale, c->st);
  }
  MF_TRY(launch_rows_r2c(x, c->cs, c->S, c->L, c->g, c->tw, false, c->st));
  MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, COL_REAL, c->P_T, nullptr, 1.f, nullptr, c->st));
  MF_TRY(launch_rows_c2r(c->S, c->L, c->g, c->tw, EPI_GRAD, out, c->cs, c->B, s, s_scale, nullptr, nullptr, nullptr,
                         nullptr, c->st));
  return MUFFIN_OK;
}

// mu_lambda = 0: gradient and the relaxed primal step of every channel in the three FFT passes;
// x is read and written in place and d goes to D.
int enqueue_local_primal(muffin_ctx* c, const float* s, float s_scale) {
  PrimalEpi pe;
  pe.D = c->D;
  pe.tau_ch = c->tau_ch;
  pe.rho = (float)c->rho;
  MF_TRY(launch_rows_r2c(c->X, c->cs, c->S, c->L, c->g, c->tw, false, c->st));
  MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, COL_REAL, c->P_T, nullptr, 1.f, nullptr, c->st));
  MF_TRY(launch_rows_c2r(c->S, c->L, c->g, c->tw, EPI_PRIMAL, c->X, c->cs, c->B, s, s_scale, nullptr, nullptr,
                         nullptr, nullptr, c->st, pe));
  return MUFFIN_OK;
}

int enqueue_spectral(muffin_ctx* c) {
  for (const Seg& s : c->segs) {
    const long long off = (long long)s.ch0 * c->cs;
    SpectralArgs a;
    a.X = c->X + off;
    a.Q = c->Q + off;
    a.V = c->V + off;
    a.D = c->D + off;
    a.W = s.W;
    a.WT = s.WT;
    a.twL = s.twL;
    a.csL = s.csL;
    a.npix = c->npix;
    a.cs = c->cs;
    a.L = s.L;
    a.use_fft = spectral_has_fft(s.L) ? 1 : 0;
    const bool blu = (c->p.flags & MUFFIN_FLAG_SPECTRAL_BLUESTEIN) ||
                     (!(c->p.flags & MUFFIN_FLAG_SPECTRAL_DENSE) && spectral_blu_default(s.L));
    a.blu = blu ? s.blu : nullptr;
    a.tau = (float)s.tau;
    a.mu_l = (float)s.mu_l;
    a.smu_l = (float)(c->sigma * s.mu_l);
    a.rho = (float)c->rho;
    MF_TRY(launch_spectral_step(a, c->st));
  }
  return MUFFIN_OK;
}

// With marks, phase boundaries are recorded in marks[0..4] and, for the second-generation
// transform, each scale's fused adjoint (marks pass 1) or analysis launch is bracketed in kev.
// par: parity of the fused tail's planes at the start of the iteration (it flips at the end).
int enqueue_iteration(muffin_ctx* c, hipEvent_t* marks, int timed_family = 0, int par = 0) {
  const long long ucs = (long long)c->np_u * c->us;
  if (marks) MF_HIP(hipEventRecord(marks[0], c->st));
  const float* s = nullptr;
  MF_TRY(enqueue_adjoint(c, c->U, c->us, ucs, c->omega_c, &s, timed_family == 1, c->fused ? c->Acar : nullptr));
  if (marks) MF_HIP(hipEventRecord(marks[1], c->st));
  if (c->local_primal) {
    MF_TRY(enqueue_local_primal(c, s, (float)c->p.mu_s));
    if (marks) MF_HIP(hipEventRecord(marks[2], c->st));
  } else {
    MF_TRY(enqueue_gradient(c, c->X, c->Q, s, (float)c->p.mu_s));
    if (marks) MF_HIP(hipEventRecord(marks[2], c->st));
    MF_TRY(enqueue_spectral(c));
  }
  if (marks) MF_HIP(hipEventRecord(marks[3], c->st));
  MF_TRY(enqueue_dual_update(c, c->D, timed_family == 2, par));
  if (marks) MF_HIP(hipEventRecord(marks[4], c->st));
  return MUFFIN_OK;
}

// Objective terms of segment si at X into dres[1..3] (data, spatial l1 unweighted by mu_s, spectral l1).
int enqueue_objective(muffin_ctx* c, int si) {
  const Seg& s = c->segs[si];
  const long long np = c->cs, off = (long long)s.ch0 * np;
  const int nch = s.L;
  float* X = c->X + off;
  MF_HIP(hipMemsetAsync(c->dres, 0, sizeof(double) * 4, c->st));
  int nb = 0;
  if (c->vis) {
    // 1/2 ||Phi x - v||^2 (one segment)
    MF_TRY(enqueue_vis_forward(c, X, np, c->vdata, -1.f, c->partial, &nb));
  } else {
    MF_TRY(launch_rows_r2c(X, np, c->S, nch, c->g, c->tw, false, c->st));
    MF_TRY(launch_cols(c->S, nch, c->g, c->tw, COL_CPLX, nullptr, c->Hhat_T + (long long)s.ch0 * c->g.pitch * c->N,
                       1.f / ((float)c->N * c->N), nullptr, c->st));
    MF_TRY(launch_rows_c2r(c->S, nch, c->g, c->tw, EPI_RESID, nullptr, np, nullptr, nullptr, 0.f, c->Y + off,
                           c->chan_w ? c->chan_w + s.ch0 : nullptr, c->partial, &nb, c->st));
  }
  MF_TRY(launch_reduce_sum(c->partial, nb, c->dres + 1, 0, c->st));
  if (c->uob) {
    MF_TRY(enqueue_uob_analysis(c, UOB_ABS, X, np, s.ch0, nch, nullptr, 0, 0, nullptr, 0, 0, 0.f, 1.f,
                                (float)(1.0 / std::sqrt((double)kUobBases)), c->dres + 2));
    MF_TRY(launch_dct_abs(X, s.WT, c->npix, np, nch, c->partial, &nb, c->st));
    return launch_reduce_sum(c->partial, nb, c->dres + 3, 0, c->st);
  }
  const float* cur = X;
  float* bufs[2] = {c->cA, c->cB};
  for (int j = 0; j < c->J; ++j) {
    float* nxt = bufs[j & 1];
    MF_TRY(launch_atrous(SM_SMOOTH, c->N, nch, j, pref(cur, np), PlaneRef{}, PlaneRef{}, pout(nxt, np), PlaneOut{},
                         0.f, 1.f, nullptr, nullptr, c->st));
    if (c->gen == 2)
      MF_TRY(launch_atrous(SM_DETAIL_ABS, c->N, nch, j, pref(nxt, np), PlaneRef{}, pref(cur, np), PlaneOut{},
                           PlaneOut{}, 0.f, 1.f, c->partial, &nb, c->st));
    else
      MF_TRY(launch_pointwise(PT_ABS_DIFF, c->N, nch, pref(nxt, np), pref(cur, np), PlaneOut{}, 0.f, 1.f, c->partial,
                              &nb, c->st));
    MF_TRY(launch_reduce_sum(c->partial, nb, c->dres + 2, 1, c->st));
    cur = nxt;
  }
  if (c->omega_c != 0.f) {
    MF_TRY(launch_pointwise(PT_ABS, c->N, nch, pref(cur, np), PlaneRef{}, PlaneOut{}, 0.f, 1.f, c->partial, &nb,
                            c->st));
    MF_TRY(launch_reduce_sum(c->partial, nb, c->dres + 2, 1, c->st));
  }
  MF_TRY(launch_dct_abs(X, s.WT, c->npix, np, nch, c->partial, &nb, c->st));
  MF_TRY(launch_reduce_sum(c->partial, nb, c->dres + 3, 0, c->st));
  return MUFFIN_OK;
}

void destroy(muffin_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  for (int k = 0; k < 2; ++k) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
  }
  void* bufs[] = {c->X, c->U, c->V, c->D, c->Q, c->B, c->Y, c->cA, c->cB, c->cT, c->S, c->Hhat_T, c->P_T,
                  c->tw, c->chan_w, c->psf_lobe, c->partial, c->dres, c->U2, c->Acar, c->tau_ch, c->Xs, c->Us, c->Vs, c->uobA, c->uobB,
                  c->vp, c->vdata, c->vpart, c->vlt, c->vnt, c->vinvn, c->XN, c->vres};
  for (Seg& s : c->segs) {
    void* sb[] = {s.W, s.WT, s.twL, s.csL, s.blu};
    for (void* b : sb)
      if (b) (void)hipFree(b);
  }
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

// n planes of np floats from src (planes sps floats apart) to dst (dps apart); waits for the copy
// when host memory is involved.
int copy_planes(float* dst, long long dps, const float* src, long long sps, long long n, long long np,
                hipMemcpyKind kind, hipStream_t st) {
  if (n <= 0) return MUFFIN_OK;
  MF_HIP(hipMemcpy2DAsync(dst, sizeof(float) * dps, src, sizeof(float) * sps, sizeof(float) * np, (size_t)n, kind,
                          st));
  if (kind != hipMemcpyDeviceToDevice) MF_HIP(hipStreamSynchronize(st));
  return MUFFIN_OK;
}
// the caller's dense [n][N][N] layout <-> the library's plane slots of ps floats (cs by default)
int planes_in(muffin_ctx* c, float* dst, const float* src, long long n, int on_device, long long ps = 0) {
  return copy_planes(dst, ps ? ps : c->cs, src, c->npix, n, c->npix,
                     on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st);
}
int planes_out(muffin_ctx* c, float* dst, const float* src, long long n, int on_device, long long ps = 0) {
  return copy_planes(dst, c->npix, src, ps ? ps : c->cs, n, c->npix,
                     on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->st);
}

// Power iterations and safety factor of beta for the visibility data term: beta is the largest
// eigenvalue of Re Phi^H Phi over all channels, estimated by power iteration from the all-ones cube
// (its estimate approaches the eigenvalue from below, hence the factor).
constexpr int kVisPowerIters = 40;
constexpr double kVisBetaMargin = 1.01;

int init_vis_data(muffin_ctx* c, const VisInit* vi);
int vis_power_beta(muffin_ctx* c, int iters, double* beta);

// Build a context over n cubes that share N, J, generation, coarse weighting, mu_s, sigma and rho
// (checked by the caller); their channels are packed one cube after the other.  With vi (one cube),
// the data term is the visibility-domain one of Sec. 2, eq. (viseq), and dirty and psf are unused.
int init_group(muffin_ctx* c, int n, const muffin_params* const* ps, const float* const* dirty,
               const float* const* psf, int on_device, const VisInit* vi = nullptr) {
  const muffin_params* p = ps[0];
  c->p = *p;
  c->vis = vi != nullptr;
  c->p.chan_weight = nullptr;
  c->N = p->N;
  c->J = p->J;
  c->gen = p->iuwt_gen;
  c->npix = (long long)p->N * p->N;
  c->cs = (c->npix + p->N + 31) / 32 * 32 + 32;
  c->us = c->npix;
  c->g = fft_geom(p->N);
  c->omega_c = p->penalize_coarse ? 1.f : 0.f;
  c->uob = p->prior == MUFFIN_PRIOR_UOB;
  c->np_u = c->uob ? kUobBases : c->J + 1;
  if (c->uob) c->uf = uob_filters();
  c->sigma = p->sigma;
  c->rho = p->rho;
  int total = 0;
  bool any_w = false;
  for (int i = 0; i < n; ++i) {
    Seg s;
    s.ch0 = total;
    s.L = ps[i]->L;
    s.mu_l = ps[i]->mu_lambda;
    total += s.L;
    any_w = any_w || ps[i]->chan_weight;
    c->segs.push_back(s);
  }
  c->L = total;
  c->cube = c->cs * total;
  c->ucube = c->us * total * c->np_u;
  c->fused_ok = !c->uob && !(p->flags & MUFFIN_FLAG_NO_FUSED_TAIL) && use_pairs(c) && c->omega_c == 1.f &&
                !iuwt_groups(c).empty() && iuwt_groups(c).back() == 2;
  c->jf = c->J - 2;
  if (c->fused_ok) {
    // default: whole-channel bands fill the GPU and a residue class is long against the halo
    int ncu = 0;
    MF_HIP(hipGetDevice(&c->device));
    MF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    c->fused = (p->flags & MUFFIN_FLAG_FUSED_TAIL) || (total >= ncu && (c->N >> c->jf) >= 64);
  }
  if (any_w) {
    c->chan_w_host.assign(total, 1.f);
    for (int i = 0; i < n; ++i)
      if (ps[i]->chan_weight)
        std::copy(ps[i]->chan_weight, ps[i]->chan_weight + ps[i]->L, c->chan_w_host.begin() + c->segs[i].ch0);
  }
  MF_HIP(hipGetDevice(&c->device));
  MF_HIP(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking));
  for (hipEvent_t* e : {&c->ev_in, &c->ev_out}) MF_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  for (hipEvent_t* e : {&c->e0, &c->e1, &c->ph[0], &c->ph[1], &c->ph[2], &c->ph[3], &c->ph[4]})
    MF_HIP(hipEventCreate(e));
  for (auto& e : c->kev) MF_HIP(hipEventCreate(&e));
  MF_TRY(fft_init_attrs(c->N));
  MF_TRY(atrous_init_attrs());
  for (const Seg& s : c->segs) MF_TRY(spectral_init_attrs(s.L));

  const long long cube = c->cube;
  const long long spec = (long long)c->L * c->N * c->g.pitch;
  MF_TRY(dalloc(&c->X, cube));
  MF_TRY(dalloc(&c->U, c->ucube));
  if (c->fused_ok) {
    MF_TRY(dalloc(&c->U2, c->us * total * 3));
    MF_TRY(dalloc(&c->Acar, cube));
  }
  MF_TRY(dalloc(&c->V, cube));
  MF_TRY(dalloc(&c->D, cube));
  MF_TRY(dalloc(&c->Q, cube));
  if (!c->vis) {
    MF_TRY(dalloc(&c->B, cube));
    MF_TRY(dalloc(&c->Y, cube));
  }
  MF_TRY(dalloc(&c->cA, cube));
  MF_TRY(dalloc(&c->cB, cube));
  MF_TRY(dalloc(&c->cT, cube));
  if (!c->vis) {
    MF_TRY(dalloc(&c->S, spec));
    MF_TRY(dalloc(&c->Hhat_T, spec));
    MF_TRY(dalloc(&c->P_T, spec));
  }
  MF_TRY(dalloc(&c->tw, c->N));
  for (Seg& s : c->segs) {
    MF_TRY(dalloc(&s.twL, s.L));
    MF_TRY(dalloc(&s.csL, s.L));
    MF_TRY(dalloc(&s.W, (long long)s.L * s.L));
    MF_TRY(dalloc(&s.WT, (long long)s.L * s.L));
    if (const int M = spectral_blu_m(s.L)) MF_TRY(dalloc(&s.blu, 2LL * M + s.L));
  }
  MF_TRY(dalloc(&c->partial, kMaxPartials));
  MF_TRY(dalloc(&c->dres, 16));
  if (!c->vis) MF_TRY(dalloc(&c->psf_lobe, c->L));
  if (c->uob) {
    MF_TRY(dalloc(&c->uobA, (long long)c->L * kUobBases * uob_cap(c, 1)));
    MF_TRY(dalloc(&c->uobB, (long long)c->L * kUobBases * uob_cap(c, 2)));
  }
  if (!c->chan_w_host.empty()) MF_TRY(dalloc(&c->chan_w, c->L));

  StreamScope scope(c);
  if (!scope.ok) return set_error("stream ordering failed"), MUFFIN_EHIP;
  hipStream_t st = c->st;
  if (c->S) MF_HIP(hipMemsetAsync(c->S, 0, sizeof(float2) * spec, st));
  MF_HIP(hipMemsetAsync(c->dres, 0, sizeof(double) * 16, st));
  // the slot padding of every cube buffer stays zero
  for (float* b : {c->X, c->V, c->D, c->Q, c->B, c->Y, c->cA, c->cB, c->cT})
    if (b) MF_HIP(hipMemsetAsync(b, 0, sizeof(float) * cube, st));
  MF_HIP(hipMemsetAsync(c->U, 0, sizeof(float) * c->ucube, st));
  if (c->fused_ok) {
    // U = 0: the carried adjoint sum of zero planes is exactly zero
    MF_HIP(hipMemsetAsync(c->U2, 0, sizeof(float) * c->us * total * 3, st));
    MF_HIP(hipMemsetAsync(c->Acar, 0, sizeof(float) * cube, st));
  }
  for (int i = 0; i < n && !c->vis; ++i) {
    const long long off = (long long)c->segs[i].ch0 * c->cs;
    MF_TRY(planes_in(c, c->Y + off, dirty[i], c->segs[i].L, on_device));
    MF_TRY(planes_in(c, c->cT + off, psf[i], c->segs[i].L, on_device));
  }
  if (c->chan_w) MF_TRY(copy_in(c->chan_w, c->chan_w_host.data(), c->L, 0, st));
  {
    auto tw = fft_twiddles(c->N);
    MF_HIP(hipMemcpyAsync(c->tw, tw.data(), sizeof(float2) * c->N, hipMemcpyHostToDevice, st));
    for (Seg& s : c->segs) {
      const int L = s.L;
      auto twl = fft_twiddles(L);
      std::vector<float2> cs(L);
      for (int k = 0; k < L; ++k) {
        const double th = M_PI * k / (2.0 * L);
        cs[k] = make_float2((float)std::cos(th), (float)std::sin(th));
      }
      std::vector<float> W((size_t)L * L), WT((size_t)L * L);
      for (int l = 0; l < L; ++l)
        for (int k = 0; k < L; ++k) {
          const double sk = (k == 0) ? std::sqrt(1.0 / L) : std::sqrt(2.0 / L);
          const double v = sk * std::cos(M_PI * (2.0 * l + 1.0) * k / (2.0 * L));
          W[(size_t)l * L + k] = (float)v;
          WT[(size_t)k * L + l] = (float)v;
        }
      MF_HIP(hipMemcpyAsync(s.twL, twl.data(), sizeof(float2) * L, hipMemcpyHostToDevice, st));
      MF_HIP(hipMemcpyAsync(s.csL, cs.data(), sizeof(float2) * L, hipMemcpyHostToDevice, st));
      MF_HIP(hipMemcpyAsync(s.W, W.data(), sizeof(float) * W.size(), hipMemcpyHostToDevice, st));
      MF_HIP(hipMemcpyAsync(s.WT, WT.data(), sizeof(float) * WT.size(), hipMemcpyHostToDevice, st));
      const std::vector<float2> blu = spectral_blu_table(L);
      if (s.blu) MF_HIP(hipMemcpyAsync(s.blu, blu.data(), sizeof(float2) * blu.size(), hipMemcpyHostToDevice, st));
      MF_HIP(hipStreamSynchronize(st));
    }
  }
  if (c->vis) {
    MF_TRY(init_vis_data(c, vi));
  } else {
  // non-finite inputs
  MF_TRY(launch_count_nonfinite(c->Y, cube, c->partial, c->dres + 0, st));
  MF_TRY(launch_count_nonfinite(c->cT, cube, c->partial, c->dres + 0, st));
  double bad = 0;
  MF_HIP(hipMemcpyAsync(&bad, c->dres, sizeof(double), hipMemcpyDeviceToHost, st));
  MF_HIP(hipStreamSynchronize(st));
  if (bad != 0) return set_error("NaN or Inf in dirty or psf"), MUFFIN_ENONFINITE;

  MF_TRY(launch_psf_lobe(c->cT, c->cs, c->psf_lobe, c->N, c->L, 4, st));
  // transfer functions: Hhat = FFT2(ifftshift(psf)), P = w |Hhat|^2 / N^2
  const float inv_n2 = 1.f / ((float)c->N * c->N);
  MF_TRY(launch_rows_r2c(c->cT, c->cs, c->S, c->L, c->g, c->tw, true, st));
  MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, COL_FWD, nullptr, nullptr, 1.f, c->Hhat_T, st));
  MF_TRY(launch_power_spectrum(c->Hhat_T, c->P_T, c->chan_w, (long long)c->g.pitch * c->N, c->L, inv_n2, st));
  // b = w H^dagger y
  MF_TRY(launch_rows_r2c(c->Y, c->cs, c->S, c->L, c->g, c->tw, false, st));
  MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, COL_CPLX_CONJ, nullptr, c->Hhat_T, inv_n2, nullptr, st));
  MF_TRY(launch_rows_c2r(c->S, c->L, c->g, c->tw, EPI_STORE, c->B, c->cs, nullptr, nullptr, 0.f, nullptr, nullptr,
                         nullptr, nullptr, st));
  if (c->chan_w) MF_TRY(launch_scale_channels(c->B, c->chan_w, c->npix, c->cs, c->L, st));
  }
  // ||W_s||^2 (FP64, shared by the group) and, per cube, beta = max_l w_l max_k |H_l(k)|^2
  // (the union of orthonormal bases divided by sqrt(8) is a tight frame: W_s^dagger W_s = I)
  if (c->uob) {
    c->Ws2 = 1.0;
  } else {
    MF_TRY(launch_frame_bound(c->N, c->J, c->gen, c->omega_c, c->partial, c->dres + 5, st));
    MF_HIP(hipMemcpyAsync(&c->Ws2, c->dres + 5, sizeof(double), hipMemcpyDeviceToHost, st));
  }
  const long long per_ch = (long long)c->g.pitch * c->N;
  for (size_t i = 0; i < c->segs.size(); ++i) {
    Seg& s = c->segs[i];
    if (c->vis) {
      MF_TRY(vis_power_beta(c, vi->d->power_iters > 0 ? vi->d->power_iters : kVisPowerIters, &s.beta));
    } else {
      MF_TRY(launch_reduce_max(c->P_T + s.ch0 * per_ch, s.L * per_ch, (double)c->N * (double)c->N, c->partial,
                               c->dres + 4, st));
      MF_HIP(hipMemcpyAsync(&s.beta, c->dres + 4, sizeof(double), hipMemcpyDeviceToHost, st));
      MF_HIP(hipStreamSynchronize(st));
    }
    s.K2 = c->p.mu_s * c->p.mu_s * c->Ws2 + s.mu_l * s.mu_l;
    s.tau = ps[i]->tau > 0 ? ps[i]->tau : 0.99 / (s.beta / 2.0 + c->sigma * s.K2);
    const double margin = 1.0 / s.tau - c->sigma * s.K2;
    if (!(margin > s.beta / 2.0))
      return set_error("step sizes violate 1/tau - sigma ||K||^2 > beta/2 (cube " + std::to_string(i) + ")"),
             MUFFIN_ESTEP;
    s.delta = 2.0 - (s.beta / 2.0) / margin;
    if (!(c->rho < s.delta)) return set_error("rho must lie in (0, delta)"), MUFFIN_ESTEP;
  }

  // the mu_lambda = 0 pass runs the primal step in the image-plane gradient's last FFT pass
  c->local_primal = !c->vis;
  for (const Seg& s : c->segs) c->local_primal = c->local_primal && s.mu_l == 0.0;
  {
    std::vector<float> tch(c->L);
    for (const Seg& s : c->segs)
      for (int l = 0; l < s.L; ++l) tch[s.ch0 + l] = (float)s.tau;
    MF_TRY(dalloc(&c->tau_ch, c->L));
    MF_HIP(hipMemcpyAsync(c->tau_ch, tch.data(), sizeof(float) * c->L, hipMemcpyHostToDevice, st));
    MF_HIP(hipStreamSynchronize(st));
  }

  MF_HIP(hipMemsetAsync(c->X, 0, sizeof(float) * cube, st));
  MF_HIP(hipMemsetAsync(c->U, 0, sizeof(float) * c->ucube, st));
  MF_HIP(hipMemsetAsync(c->V, 0, sizeof(float) * cube, st));
  MF_HIP(hipMemsetAsync(c->D, 0, sizeof(float) * cube, st));
  MF_HIP(hipStreamSynchronize(st));
  return MUFFIN_OK;
}

// Tables and data of the visibility data term (Sec. 2, eq. (viseq)): pixel (i, j) sits at
// l = (j - N/2) cell, m = (i - N/2) cell, n = sqrt(1 - l^2 - m^2) (FP64 on the host); each channel's
// baselines are divided by its wavelength in FP64.
int init_vis_data(muffin_ctx* c, const VisInit* vi) {
  const muffin_vis_desc* d = vi->d;
  const int N = c->N, L = c->L, K = d->K;
  const long long LK = (long long)L * K, np = c->npix;
  c->K = K;
  c->vC = vis_chunks(N, K, L);
  MF_TRY(dalloc(&c->vp, LK));
  MF_TRY(dalloc(&c->vdata, LK));
  MF_TRY(dalloc(&c->vpart, (long long)c->vC * LK));
  MF_TRY(dalloc(&c->vlt, N));
  MF_TRY(dalloc(&c->vnt, np));
  MF_TRY(dalloc(&c->vinvn, np));
  MF_TRY(dalloc(&c->XN, np * L));
  std::vector<double> lt(N), nt(np);
  std::vector<float> invn(np);
  for (int j = 0; j < N; ++j) lt[j] = (j - N / 2) * d->cell;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double n = std::sqrt(1.0 - lt[j] * lt[j] - lt[i] * lt[i]);
      nt[(size_t)i * N + j] = n;
      invn[(size_t)i * N + j] = (float)(1.0 / n);
    }
  std::vector<VisPt> vp(LK);
  for (int l = 0; l < L; ++l)
    for (int k = 0; k < K; ++k) {
      VisPt& q = vp[(size_t)l * K + k];
      q.u = d->uvw[3 * k] / d->lambda[l];
      q.v = d->uvw[3 * k + 1] / d->lambda[l];
      q.w = d->uvw[3 * k + 2] / d->lambda[l];
      q.rre = q.rim = 0.f;
    }
  hipStream_t st = c->st;
  MF_HIP(hipMemcpyAsync(c->vlt, lt.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
  MF_HIP(hipMemcpyAsync(c->vnt, nt.data(), sizeof(double) * np, hipMemcpyHostToDevice, st));
  MF_HIP(hipMemcpyAsync(c->vinvn, invn.data(), sizeof(float) * np, hipMemcpyHostToDevice, st));
  MF_HIP(hipMemcpyAsync(c->vp, vp.data(), sizeof(VisPt) * LK, hipMemcpyHostToDevice, st));
  MF_TRY(copy_in((float*)c->vdata, vi->vis, (size_t)(2 * LK), vi->on_device, st));
  MF_HIP(hipMemsetAsync(c->dres, 0, sizeof(double), st));
  MF_TRY(launch_count_nonfinite((const float*)c->vdata, 2 * LK, c->partial, c->dres + 0, st));
  double bad = 0;
  MF_HIP(hipMemcpyAsync(&bad, c->dres, sizeof(double), hipMemcpyDeviceToHost, st));
  MF_HIP(hipStreamSynchronize(st));  // also keeps the host tables alive until their copies are done
  if (bad != 0) return set_error("NaN or Inf in the visibilities"), MUFFIN_ENONFINITE;
  return MUFFIN_OK;
}

// beta = kVisBetaMargin ||A x_T|| after `iters` steps x <- A x / ||A x|| from the all-ones cube,
// A = Re Phi^H Phi over every channel (norms in FP64).  Uses the scratch planes cT and cA.
int vis_power_beta(muffin_ctx* c, int iters, double* beta) {
  hipStream_t st = c->st;
  const long long np = c->npix;
  float* x = c->cT;
  float* y = c->cA;
  {
    std::vector<float> ones((size_t)(np * c->L), 1.f);
    MF_TRY(planes_in(c, x, ones.data(), c->L, 0));
  }
  MF_TRY(launch_vis_scale(x, c->cs, c->N, c->L, (float)(1.0 / std::sqrt((double)np * c->L)), st));
  double est = 0.0;
  for (int t = 0; t < iters; ++t) {
    MF_TRY(enqueue_vis_forward(c, x, c->cs, nullptr, 0.f, nullptr, nullptr));
    MF_TRY(launch_vis_adj(c->vp, c->K, c->L, c->vlt, c->vnt, c->vinvn, c->N, y, c->cs, nullptr, 0, 0.f, st));
    MF_TRY(launch_diff_norms(y, c->cs, nullptr, 0, np, c->L, c->partial, c->dres + 6, c->dres + 7, 0, st));
    double ss = 0.0;
    MF_HIP(hipMemcpyAsync(&ss, c->dres + 7, sizeof(double), hipMemcpyDeviceToHost, st));
    MF_HIP(hipStreamSynchronize(st));
    if (!(ss > 0.0) || !std::isfinite(ss)) return set_error("beta: the power iteration broke down"), MUFFIN_ENONFINITE;
    est = std::sqrt(ss);
    MF_TRY(launch_vis_scale(y, c->cs, c->N, c->L, (float)(1.0 / est), st));
    std::swap(x, y);
  }
  *beta = kVisBetaMargin * est;
  return MUFFIN_OK;
}

// Before a monitored iteration: X, U (the planes of the current parity, into dense planes) and V
// are copied aside (the copies are allocated on first use).
int snapshot_state(muffin_ctx* c) {
  const long long np = c->npix, J1 = c->np_u;
  if (!c->Xs) MF_TRY(dalloc(&c->Xs, c->cube));
  if (!c->Vs) MF_TRY(dalloc(&c->Vs, c->cube));
  if (!c->Us) MF_TRY(dalloc(&c->Us, (long long)c->L * J1 * np));
  MF_HIP(hipMemcpyAsync(c->Xs, c->X, sizeof(float) * c->cube, hipMemcpyDeviceToDevice, c->st));
  MF_HIP(hipMemcpyAsync(c->Vs, c->V, sizeof(float) * c->cube, hipMemcpyDeviceToDevice, c->st));
  for (int k = 0; k < c->np_u; ++k) {
    const PlaneOut u = uplane(c, k, c->upar);
    MF_TRY(copy_planes(c->Us + k * np, J1 * np, u.p, u.cs, c->L, np, hipMemcpyDeviceToDevice, c->st));
  }
  return MUFFIN_OK;
}

// After it: out = {||X - Xs||, ||X||, ||U - Us||, ||U||, ||V - Vs||, ||V||} (FP64, L2 over the cube).
int state_change(muffin_ctx* c, double out[6]) {
  const long long np = c->npix, J1 = c->np_u;
  MF_TRY(launch_diff_norms(c->X, c->cs, c->Xs, c->cs, np, c->L, c->partial, c->dres + 6, c->dres + 7, 0, c->st));
  for (int k = 0; k < c->np_u; ++k) {
    const PlaneOut u = uplane(c, k, c->upar);
    MF_TRY(launch_diff_norms(u.p, u.cs, c->Us + k * np, J1 * np, np, c->L, c->partial, c->dres + 8, c->dres + 9,
                             k > 0, c->st));
  }
  MF_TRY(launch_diff_norms(c->V, c->cs, c->Vs, c->cs, np, c->L, c->partial, c->dres + 10, c->dres + 11, 0, c->st));
  double h[6];
  MF_HIP(hipMemcpyAsync(h, c->dres + 6, sizeof(h), hipMemcpyDeviceToHost, c->st));
  MF_HIP(hipStreamSynchronize(c->st));
  for (int i = 0; i < 6; ++i) out[i] = std::sqrt(h[i]);
  return MUFFIN_OK;
}

// SNR of the channels [ch0, ch0 + nch) of X against a dense truth cube (Sec. 4):
// 10 log10(||X*||^2 / ||X - X*||^2); the truth is staged in the scratch planes cT.
int snr_of(muffin_ctx* c, int ch0, int nch, const float* truth, int on_device, double* snr) {
  const long long np = c->npix, off = (long long)ch0 * c->cs;
  MF_TRY(copy_planes(c->cT + off, c->cs, truth, np, nch, np,
                     on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st));
  MF_TRY(launch_diff_norms(c->cT + off, c->cs, c->X + off, c->cs, np, nch, c->partial, c->dres + 12, c->dres + 13, 0,
                           c->st));
  double h[2];
  MF_HIP(hipMemcpyAsync(h, c->dres + 12, sizeof(h), hipMemcpyDeviceToHost, c->st));
  MF_HIP(hipStreamSynchronize(c->st));
  *snr = 10.0 * std::log10(h[1] / h[0]);
  return MUFFIN_OK;
}

// Capture one iteration into a graph per parity of the fused tail's planes (capture records the
// work without running it).
int ensure_graph(muffin_ctx* c) {
  for (int par = 0; par < (c->fused ? 2 : 1); ++par) {
    if (c->gexec[par]) continue;
    MF_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_iteration(c, nullptr, 0, par);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(c->st, &gr);
    if (rc != MUFFIN_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    MF_HIP(e);
    c->graph[par] = gr;
    MF_HIP(hipGraphInstantiate(&c->gexec[par], c->graph[par], nullptr, nullptr, 0));
  }
  return MUFFIN_OK;
}

void drop_graphs(muffin_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
}

// Switch the fused tail on or off between iterations: its planes go back to U when it is switched
// off while they are in U2, and the carried sum is rebuilt when it is switched on.
int set_fused(muffin_ctx* c, bool on) {
  if (on == c->fused) return MUFFIN_OK;
  if (on && !c->fused_ok) return set_error("fused tail not available for this context"), MUFFIN_EINVAL;
  if (!on && c->upar) {
    const long long np = c->npix;
    MF_TRY(copy_planes(c->U + (long long)c->jf * c->us, c->np_u * c->us, c->U2, 3 * c->us, c->L, 3 * np,
                       hipMemcpyDeviceToDevice, c->st));
    c->upar = 0;
  }
  if (on) c->acar_ok = false;
  c->fused = on;
  drop_graphs(c);
  return MUFFIN_OK;
}

// Before iterating: with a fused tail, the carried adjoint sum must match the current planes (it
// does unless U was set from outside); recompute it with the plain adjoint pair if not.
int ensure_carry(muffin_ctx* c) {
  if (!c->fused || c->acar_ok) return MUFFIN_OK;
  const int j = c->jf, par = c->upar;
  MF_TRY(launch_pair(PR_ADJOINT, c->N, c->L, j, uref(c, j + 1, par), uref(c, j, par), uref(c, c->J, par),
                     pout(c->Acar, c->cs), PlaneOut{}, PlaneOut{}, 0.f, 1.f, 0.f, c->st));
  c->acar_ok = true;
  return MUFFIN_OK;
}

// n iterations by graph replay, the parity of the fused tail's planes flipping after each.
int replay(muffin_ctx* c, int n) {
  MF_TRY(ensure_carry(c));
  for (int i = 0; i < n; ++i) {
    MF_HIP(hipGraphLaunch(c->gexec[c->upar], c->st));
    if (c->fused) c->upar ^= 1;
  }
  return MUFFIN_OK;
}

// Autotuner: for every band, pair, triple or fused launch of the iteration, time each band height
// that divides N with each split of a band's residue classes over 1, 2, 4 or 8 workgroups (up to
// 2^j) on the context's own sizes (reading state, writing only scratch planes) and keep the fastest.
int autotune(muffin_ctx* c, int reps, std::string& rep) {
  if (c->uob) {
    rep += "{\"N\": " + std::to_string(c->N) + ", \"channels\": " + std::to_string(c->L) +
           ", \"prior\": \"union of bases\", \"scales\": []}";
    return MUFFIN_OK;
  }
  const long long np = c->cs, us = c->us, ucs = (long long)c->np_u * us;
  // the schedule without the fused tail, plus the fused launch when it is available; the faster
  // of the fused launch and the two it replaces is kept
  const bool was_fused = c->fused;
  c->fused = false;
  std::vector<IuwtStep> sched = analysis_schedule(c);
  for (const IuwtStep& st : adjoint_schedule(c)) sched.push_back(st);
  c->fused = was_fused;
  if (c->fused_ok) sched.push_back({PR_FUSED, c->jf, "analysis pair + next adjoint pair"});
  double t_fused = 0, t_an = 0, t_adj = 0;
  rep += "{\"N\": " + std::to_string(c->N) + ", \"channels\": " + std::to_string(c->L) + ", \"scales\": [";
  bool firstrep = true;
  for (const IuwtStep& L : sched) {
    const int mode = L.mode, j = L.j;
    double best = 1e30;
    int best_ty = atrous_band_rows(c->N, j, mode, c->L), best_cg = atrous_class_groups(c->N, j, mode, c->L);
    const int max_cg = std::min(1 << j, 8);
    std::vector<std::pair<int, int>> tiles;  // (band rows, class groups)
    for (int TY = 16; TY <= c->N; TY *= 2)
      if (c->N % TY == 0)
        for (int cg = 1; cg <= max_cg; cg *= 2) tiles.push_back({TY, cg});
    std::string cand;
    for (const auto& [TY, cg] : tiles) {
      MF_TRY(atrous_set_band_rows(c->N, j, mode, TY));
      MF_TRY(atrous_set_class_groups(c->N, j, mode, cg));
      auto launch = [&]() -> int {
        switch (mode) {
          case PR_FUSED:
            return launch_fused_pair(c->N, c->L, j, pref(c->X, np), uref(c, j, c->upar), uref(c, j + 1, c->upar),
                                     uref(c, c->J, c->upar), pout(c->cB, np), pout(c->cT, np), pout(c->cA, np),
                                     pout(c->D, np), 0.f, 1.f, 0.f, c->st, 1);
          case PR_ANALYSIS:
          case PR_ANALYSIS_C:
          case P1_ANALYSIS:
          case P1_ANALYSIS_C:
            return launch_pair(mode, c->N, c->L, j, pref(c->X, np), PlaneRef{}, PlaneRef{}, pout(c->cB, np),
                               pout(c->cT, np), pout(c->cA, np), 0.f, 1.f, 0.f, c->st, 1);
          case TR_ANALYSIS:
          case TR_ANALYSIS_C:
            return launch_triple(mode, c->N, c->L, j, pref(c->X, np), PlaneRef{}, PlaneRef{}, PlaneRef{},
                                 pout(c->cB, np), pout(c->cT, np), pout(c->cA, np), pout(c->D, np), 0.f, 1.f, 0.f,
                                 c->st, 1);
          case TR_ADJOINT:
            return launch_triple(mode, c->N, c->L, j, pref(c->U + (long long)(j + 2) * us, ucs),
                                 pref(c->U + (long long)(j + 1) * us, ucs), pref(c->U + (long long)j * us, ucs),
                                 pref(c->cA, np), pout(c->cB, np), PlaneOut{}, PlaneOut{}, PlaneOut{}, 0.f, 1.f, 0.f,
                                 c->st, 1);
          case PR_ADJOINT:
          case P1_ADJOINT:
            return launch_pair(mode, c->N, c->L, j, pref(c->U + (long long)(j + 1) * us, ucs),
                               pref(c->U + (long long)j * us, ucs), pref(c->cA, np), pout(c->cB, np), PlaneOut{},
                               PlaneOut{}, 0.f, 1.f, 0.f, c->st, 1);
          case DB_ADJOINT:
            return launch_atrous(mode, c->N, c->L, j, pref(c->U + (long long)j * us, ucs), pref(c->cA, np),
                                 pref(c->cA, np), pout(c->cB, np), PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st, 1);
          case SM_SUBADD:
            return launch_atrous(mode, c->N, c->L, j, pref(c->cA, np), pref(c->cA, np), pref(c->cA, np),
                                 pout(c->cB, np), PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st, 1);
          default:  // analysis kernels of one scale
            return launch_atrous(mode, c->N, c->L, j, pref(c->X, np), PlaneRef{}, PlaneRef{}, pout(c->cB, np),
                                 pout(c->cT, np), 0.f, 1.f, nullptr, nullptr, c->st, 1, 0.f);
        }
      };
      MF_TRY(launch());
      MF_HIP(hipEventRecord(c->e0, c->st));
      for (int r = 0; r < reps; ++r) MF_TRY(launch());
      MF_HIP(hipEventRecord(c->e1, c->st));
      MF_HIP(hipEventSynchronize(c->e1));
      float tm = 0.f;
      MF_HIP(hipEventElapsedTime(&tm, c->e0, c->e1));
      const double ms = tm / reps;
      if (!cand.empty()) cand += ", ";
      cand += "\"" + std::to_string(TY) + "x" + std::to_string(cg) + "\": " + std::to_string(ms);
      if (ms < best) {
        best = ms;
        best_ty = TY;
        best_cg = cg;
      }
    }
    MF_TRY(atrous_set_band_rows(c->N, j, mode, best_ty));
    MF_TRY(atrous_set_class_groups(c->N, j, mode, best_cg));
    if (mode == PR_FUSED) t_fused = best;
    if (mode == PR_ANALYSIS_C && j == c->jf) t_an = best;
    if (mode == PR_ADJOINT && j == c->jf) t_adj = best;
    if (!firstrep) rep += ", ";
    firstrep = false;
    rep += "{\"j\": " + std::to_string(j) + ", \"kernel\": \"" + L.name + "\", \"family\": " +
           std::to_string(atrous_class(mode)) + ", \"rows\": " +
           std::to_string(best_ty) + ", \"class_groups\": " + std::to_string(best_cg) + ", \"ms\": " + std::to_string(best) + ", \"candidates_ms\": {" + cand + "}}";
  }
  rep += "]";
  if (c->fused_ok) {
    if (!(c->p.flags & MUFFIN_FLAG_FUSED_TAIL)) MF_TRY(set_fused(c, t_fused < t_an + t_adj));
    rep += std::string(", \"fused_tail\": ") + (c->fused ? "true" : "false") +
           ", \"fused_ms\": " + std::to_string(t_fused) + ", \"separate_ms\": " + std::to_string(t_an + t_adj);
  }
  rep += "}";
  // recapture the iteration with the chosen tiles
  drop_graphs(c);
  return MUFFIN_OK;
}

int write_report(const std::string& rep, char* out, size_t len) {
  if (!out || len == 0) return MUFFIN_OK;
  const size_t n = rep.size() < len - 1 ? rep.size() : len - 1;
  std::memcpy(out, rep.data(), n);
  out[n] = 0;
  return MUFFIN_OK;
}

constexpr uint64_t kMagic = 0x4d5546464e434b31ull;  // "MUFFNCK1"
// The header's kind field: the spatial prior, plus 0x100 for a context with the visibility data term
// (a state written by one kind of context is rejected by the other).
static int32_t blob_kind(const muffin_ctx* c) { return c->p.prior | (c->vis ? 0x100 : 0); }
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

int muffin_uob_filter(int32_t n, double* h, int32_t len) { return uob_lowpass(n, h, len); }

int muffin_debug_oob(uint64_t* count) {
  if (!count) return mf::set_error("debug_oob: count is NULL"), MUFFIN_EINVAL;
#ifdef MF_CHECKED
  unsigned long long total = 0, n = 0;
  for (int (*take)(unsigned long long*) : {mf::oob_take_fft, mf::oob_take_iuwt, mf::oob_take_spectral,
                                           mf::oob_take_uob, mf::oob_take_vis}) {
    MF_TRY(take(&n));
    total += n;
  }
  *count = total;
  return MUFFIN_OK;
#else
  *count = 0;
  return mf::set_error("debug_oob: not a checked build (MF_CHECKED)"), MUFFIN_EINVAL;
#endif
}

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
  const int rc = init_group(c, 1, &p, &dirty, &psf, inputs_on_device);
  if (rc != MUFFIN_OK) {
    destroy(c);
    return rc;
  }
  *out = c;
  return MUFFIN_OK;
}

int muffin_init_vis(muffin_ctx** out, const muffin_params* p, const muffin_vis_desc* d, const float* vis,
                    int vis_on_device, void* hip_stream) {
  if (!out) return set_error("out is NULL"), MUFFIN_EINVAL;
  *out = nullptr;
  MF_TRY(validate(p));
  if (!d || !vis || !d->uvw || !d->lambda) return set_error("desc, vis, uvw or lambda is NULL"), MUFFIN_EINVAL;
  if (p->N % 8) return set_error("the visibility data term needs N to be a multiple of 8"), MUFFIN_EINVAL;
  if (d->K < 1 || d->K > (1 << 22)) return set_error("K must be in [1, 2^22]"), MUFFIN_EINVAL;
  if (d->power_iters < 0 || d->power_iters > 100000) return set_error("power_iters must be in [0, 1e5]"), MUFFIN_EINVAL;
  const double half = 0.5 * p->N * d->cell;
  if (!(d->cell > 0) || !std::isfinite(d->cell) || !(2.0 * half * half < 1.0))
    return set_error("cell must be > 0 with every pixel inside the unit disc (l^2 + m^2 < 1)"), MUFFIN_EINVAL;
  for (int l = 0; l < p->L; ++l)
    if (!(d->lambda[l] > 0) || !std::isfinite(d->lambda[l]))
      return set_error("every wavelength must be finite and > 0"), MUFFIN_EINVAL;
  for (long long i = 0; i < 3LL * d->K; ++i)
    if (!std::isfinite(d->uvw[i])) return set_error("NaN or Inf in uvw"), MUFFIN_ENONFINITE;
  muffin_ctx* c = new (std::nothrow) muffin_ctx();
  if (!c) return set_error("host allocation failed"), MUFFIN_ENOMEM;
  c->user = (hipStream_t)hip_stream;
  const VisInit vi{d, vis, vis_on_device};
  const int rc = init_group(c, 1, &p, nullptr, nullptr, 0, &vi);
  if (rc != MUFFIN_OK) {
    destroy(c);
    return rc;
  }
  *out = c;
  return MUFFIN_OK;
}

int muffin_vis_residual(muffin_ctx* c, float* r, int on_device) {
  if (!c || !r) return set_error("bad arguments"), MUFFIN_EINVAL;
  if (!c->vis) return set_error("not a visibility context"), MUFFIN_EINVAL;
  StreamScope scope(c);
  // L K complex values: written straight into a device buffer, or staged for a host one (the
  // scratch planes hold L (N^2 + N + 32) floats, too few for K above about N^2 / 2)
  float2* dst = reinterpret_cast<float2*>(r);
  if (!on_device) {
    if (!c->vres) MF_TRY(dalloc(&c->vres, (size_t)c->L * c->K));
    dst = c->vres;
  }
  MF_TRY(enqueue_vis_forward(c, c->X, c->cs, c->vdata, -1.f, nullptr, nullptr, dst));
  if (on_device) return MUFFIN_OK;
  return copy_out(r, reinterpret_cast<const float*>(c->vres), (size_t)(2LL * c->L * c->K), 0, c->st);
}

void muffin_free(muffin_ctx* c) { destroy(c); }

int muffin_set_band_tiles(int32_t N, int32_t j, int32_t family, int32_t rows, int32_t class_groups) {
  if (N < 1 || N > 1024 || j < 0 || j > 10) return mf::set_error("set_band_tiles: N or j out of range"), MUFFIN_EINVAL;
  return mf::atrous_set_tiles(N, j, family, rows, class_groups);
}

int muffin_autotune(muffin_ctx* c, int32_t reps, char* report, size_t report_len) {
  if (!c || reps < 1) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  std::string rep;
  MF_TRY(autotune(c, reps, rep));
  return write_report(rep, report, report_len);
}

// ---------------------------------------------------------------------------------- batches
struct muffin_batch {
  std::vector<muffin_ctx*> groups;
  std::vector<std::pair<int, int>> map;  // cube -> (group, segment)
  hipStream_t user = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

void muffin_batch_free(muffin_batch* b) {
  if (!b) return;
  for (muffin_ctx* g : b->groups) destroy(g);
  if (b->e0) (void)hipEventDestroy(b->e0);
  if (b->e1) (void)hipEventDestroy(b->e1);
  delete b;
}

int muffin_batch_init(muffin_batch** out, int32_t n_cubes, const muffin_params* p, const float* const* dirty,
                      const float* const* psf, int inputs_on_device, void* hip_stream) {
  if (!out) return set_error("out is NULL"), MUFFIN_EINVAL;
  *out = nullptr;
  if (n_cubes < 1 || !p || !dirty || !psf) return set_error("bad arguments"), MUFFIN_EINVAL;
  for (int i = 0; i < n_cubes; ++i) {
    MF_TRY(validate(p + i));
    if (!dirty[i] || !psf[i]) return set_error("dirty or psf is NULL"), MUFFIN_EINVAL;
  }
  muffin_batch* b = new (std::nothrow) muffin_batch();
  if (!b) return set_error("host allocation failed"), MUFFIN_ENOMEM;
  b->user = (hipStream_t)hip_stream;
  b->map.assign(n_cubes, {-1, -1});
  auto fail = [&](int rc) {
    muffin_batch_free(b);
    return rc;
  };
  if (hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess)
    return fail((set_error("event creation failed"), MUFFIN_EHIP));
  // group cubes that can share the per-channel phases
  auto same = [&](const muffin_params& a, const muffin_params& c) {
    return a.N == c.N && a.J == c.J && a.iuwt_gen == c.iuwt_gen && a.penalize_coarse == c.penalize_coarse &&
           a.prior == c.prior &&
           a.mu_s == c.mu_s && a.sigma == c.sigma && a.rho == c.rho && a.flags == c.flags;
  };
  std::vector<char> done(n_cubes, 0);
  for (int i = 0; i < n_cubes; ++i) {
    if (done[i]) continue;
    std::vector<int> idx;
    for (int k = i; k < n_cubes; ++k)
      if (!done[k] && same(p[i], p[k])) {
        idx.push_back(k);
        done[k] = 1;
      }
    std::vector<const muffin_params*> ps;
    std::vector<const float*> ds, fs;
    for (int k : idx) {
      ps.push_back(p + k);
      ds.push_back(dirty[k]);
      fs.push_back(psf[k]);
    }
    muffin_ctx* g = new (std::nothrow) muffin_ctx();
    if (!g) return fail((set_error("host allocation failed"), MUFFIN_ENOMEM));
    g->user = b->user;
    const int rc = init_group(g, (int)idx.size(), ps.data(), ds.data(), fs.data(), inputs_on_device);
    if (rc != MUFFIN_OK) {
      destroy(g);
      return fail(rc);
    }
    for (size_t s = 0; s < idx.size(); ++s) b->map[idx[s]] = {(int)b->groups.size(), (int)s};
    b->groups.push_back(g);
  }
  *out = b;
  return MUFFIN_OK;
}

// All groups replay their graphs concurrently, each on its own stream, between two events of the
// caller's stream.
static int batch_run(muffin_batch* b, int n_iter, double* ms) {
  MF_HIP(hipEventRecord(b->e0, b->user));
  for (muffin_ctx* g : b->groups) {
    MF_HIP(hipStreamWaitEvent(g->st, b->e0, 0));
    MF_TRY(ensure_graph(g));
    MF_TRY(replay(g, n_iter));
    MF_HIP(hipEventRecord(g->ev_out, g->st));
    g->iter += n_iter;
  }
  for (muffin_ctx* g : b->groups) MF_HIP(hipStreamWaitEvent(b->user, g->ev_out, 0));
  MF_HIP(hipEventRecord(b->e1, b->user));
  if (ms) {
    MF_HIP(hipEventSynchronize(b->e1));
    float t = 0.f;
    MF_HIP(hipEventElapsedTime(&t, b->e0, b->e1));
    *ms = t;
  }
  return MUFFIN_OK;
}

int muffin_batch_step(muffin_batch* b, int32_t n_iter) {
  if (!b || n_iter < 0) return set_error("bad arguments"), MUFFIN_EINVAL;
  return n_iter ? batch_run(b, n_iter, nullptr) : MUFFIN_OK;
}

int muffin_batch_step_timed(muffin_batch* b, int32_t n_iter, double* ms) {
  if (!b || !ms || n_iter < 1) return set_error("bad arguments"), MUFFIN_EINVAL;
  // capture every group's graph first so that capture stays out of the timed region
  for (muffin_ctx* g : b->groups) MF_TRY(ensure_graph(g));
  return batch_run(b, n_iter, ms);
}

static int batch_cube(muffin_batch* b, int32_t cube, muffin_ctx** g, int* si) {
  if (!b || cube < 0 || cube >= (int)b->map.size()) return set_error("bad cube index"), MUFFIN_EINVAL;
  *g = b->groups[b->map[cube].first];
  *si = b->map[cube].second;
  return MUFFIN_OK;
}

int muffin_batch_objective(muffin_batch* b, int32_t cube, double out[4]) {
  muffin_ctx* g;
  int si;
  MF_TRY(batch_cube(b, cube, &g, &si));
  if (!out) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(g);
  MF_TRY(enqueue_objective(g, si));
  double h[4];
  MF_HIP(hipMemcpyAsync(h, g->dres, sizeof(h), hipMemcpyDeviceToHost, g->st));
  MF_HIP(hipStreamSynchronize(g->st));
  out[1] = h[1];
  out[2] = g->p.mu_s * h[2];
  out[3] = g->segs[si].mu_l * h[3];
  out[0] = out[1] + out[2] + out[3];
  if (!std::isfinite(out[0])) return set_error("objective is not finite"), MUFFIN_ENONFINITE;
  return MUFFIN_OK;
}

int muffin_batch_set_x(muffin_batch* b, int32_t cube, const float* x0, int on_device) {
  muffin_ctx* g;
  int si;
  MF_TRY(batch_cube(b, cube, &g, &si));
  if (!x0) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(g);
  const Seg& s = g->segs[si];
  const long long off = (long long)s.ch0 * g->cs, J1 = g->np_u;
  MF_TRY(planes_in(g, g->X + off, x0, s.L, on_device));
  MF_TRY(launch_clamp_pos(g->X + off, (long long)s.L * g->cs, g->st));
  // this cube's duals: U (both buffers of the fused tail's planes) and V; the carried adjoint sum
  // of zero planes is zero, so its rows for these channels stay consistent
  MF_HIP(hipMemsetAsync(g->U + (long long)s.ch0 * J1 * g->us, 0, sizeof(float) * s.L * J1 * g->us, g->st));
  if (g->U2) MF_HIP(hipMemsetAsync(g->U2 + (long long)s.ch0 * 3 * g->us, 0, sizeof(float) * s.L * 3 * g->us, g->st));
  if (g->Acar) MF_HIP(hipMemsetAsync(g->Acar + off, 0, sizeof(float) * s.L * g->cs, g->st));
  MF_HIP(hipMemsetAsync(g->V + off, 0, sizeof(float) * s.L * g->cs, g->st));
  return MUFFIN_OK;
}

int muffin_batch_warm_input(muffin_batch* b, int32_t cube, float* out, int on_device) {
  muffin_ctx* g;
  int si;
  MF_TRY(batch_cube(b, cube, &g, &si));
  if (!out) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(g);
  const Seg& s = g->segs[si];
  MF_TRY(cnn_warm_input(g->Y + (long long)s.ch0 * g->cs, g->cs, g->psf_lobe + s.ch0, g->cA, g->N, s.L, g->st));
  return copy_out(out, g->cA, (size_t)(g->npix * s.L), on_device, g->st);
}

int muffin_batch_snr(muffin_batch* b, int32_t cube, const float* truth, int on_device, double* snr_db) {
  muffin_ctx* g;
  int si;
  MF_TRY(batch_cube(b, cube, &g, &si));
  if (!truth || !snr_db) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(g);
  return snr_of(g, g->segs[si].ch0, g->segs[si].L, truth, on_device, snr_db);
}

int muffin_batch_get_x(muffin_batch* b, int32_t cube, float* x, int on_device) {
  muffin_ctx* g;
  int si;
  MF_TRY(batch_cube(b, cube, &g, &si));
  if (!x) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(g);
  const Seg& s = g->segs[si];
  return planes_out(g, x, g->X + (long long)s.ch0 * g->cs, s.L, on_device);
}

int muffin_batch_info(muffin_batch* b, int32_t cube, double out[8]) {
  muffin_ctx* g;
  int si;
  MF_TRY(batch_cube(b, cube, &g, &si));
  if (!out) return set_error("bad arguments"), MUFFIN_EINVAL;
  const Seg& s = g->segs[si];
  out[0] = s.tau;
  out[1] = g->sigma;
  out[2] = g->rho;
  out[3] = s.beta;
  out[4] = s.K2;
  out[5] = g->Ws2;
  out[6] = s.delta;
  out[7] = (double)g->iter;
  return MUFFIN_OK;
}

int muffin_batch_autotune(muffin_batch* b, int32_t reps, char* report, size_t report_len) {
  if (!b || reps < 1) return set_error("bad arguments"), MUFFIN_EINVAL;
  std::string rep = "[";
  for (size_t i = 0; i < b->groups.size(); ++i) {
    StreamScope scope(b->groups[i]);
    if (i) rep += ", ";
    MF_TRY(autotune(b->groups[i], reps, rep));
  }
  rep += "]";
  return write_report(rep, report, report_len);
}

int muffin_step(muffin_ctx* c, int32_t n_iter) {
  if (!c || n_iter < 0) return set_error("bad context or n_iter"), MUFFIN_EINVAL;
  if (n_iter == 0) return MUFFIN_OK;
  StreamScope scope(c);
  if (!scope.ok) return set_error("stream ordering failed"), MUFFIN_EHIP;
  MF_TRY(ensure_graph(c));
  MF_TRY(replay(c, n_iter));
  c->iter += n_iter;
  return MUFFIN_OK;
}

int muffin_step_timed(muffin_ctx* c, int32_t n_iter, double* ms) {
  if (!c || !ms || n_iter < 1) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  if (!scope.ok) return set_error("stream ordering failed"), MUFFIN_EHIP;
  MF_TRY(ensure_graph(c));
  MF_TRY(ensure_carry(c));
  MF_HIP(hipEventRecord(c->e0, c->st));
  MF_TRY(replay(c, n_iter));
  MF_HIP(hipEventRecord(c->e1, c->st));
  MF_HIP(hipEventSynchronize(c->e1));
  float t = 0.f;
  MF_HIP(hipEventElapsedTime(&t, c->e0, c->e1));
  *ms = t;
  c->iter += n_iter;
  return MUFFIN_OK;
}

int muffin_profile(muffin_ctx* c, int32_t n_iter, double ms[32]) {
  if (!c || !ms || n_iter < 1) return set_error("bad arguments"), MUFFIN_EINVAL;
  for (int i = 0; i < 32; ++i) ms[i] = 0;
  StreamScope scope(c);
  double ksum[K_KINDS] = {};
  int kcnt[K_KINDS] = {}, fam_iters[3] = {0, 0, 0};
  MF_TRY(ensure_carry(c));
  for (int it = 0; it < n_iter; ++it) {
    // alternate which kernel family is bracketed so the marks do not pile up in one iteration
    const int fam = c->gen == 2 ? 1 + (it & 1) : 0;
    c->nk = 0;
    MF_TRY(enqueue_iteration(c, c->ph, fam, c->upar));
    if (c->fused) c->upar ^= 1;
    MF_HIP(hipEventSynchronize(c->ph[4]));
    float tph[4];
    for (int k = 0; k < 4; ++k) MF_HIP(hipEventElapsedTime(&tph[k], c->ph[k], c->ph[k + 1]));
    for (int k = 0; k < 4; ++k) {
      ms[k + 1] += tph[k] / n_iter;
      ms[0] += tph[k] / n_iter;
    }
    for (int i = 0; i < c->nk; ++i) {
      float tk = 0.f;
      MF_HIP(hipEventElapsedTime(&tk, c->kev[2 * i], c->kev[2 * i + 1]));
      ksum[c->kkind[i]] += tk;
      ++kcnt[c->kkind[i]];
    }
    ++fam_iters[fam];
  }
  c->nk = 0;
  for (int k = 0; k < K_KINDS; ++k) {
    if (!kcnt[k]) continue;
    const int fam = (k == K_DB_ADJOINT || k == K_PR_ADJOINT || k == K_TR_ADJOINT) ? 1 : 2;
    ms[8 + 2 * k] = ksum[k] / kcnt[k];
    ms[9 + 2 * k] = fam_iters[fam] ? (double)kcnt[k] / fam_iters[fam] : 0.0;
  }
  c->iter += n_iter;
  return MUFFIN_OK;
}

int muffin_objective(muffin_ctx* c, double out[4]) {
  if (!c || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  MF_TRY(enqueue_objective(c, 0));
  double h[4];
  MF_HIP(hipMemcpyAsync(h, c->dres, sizeof(h), hipMemcpyDeviceToHost, c->st));
  MF_HIP(hipStreamSynchronize(c->st));
  out[1] = h[1];
  out[2] = c->p.mu_s * h[2];
  out[3] = c->segs[0].mu_l * h[3];
  out[0] = out[1] + out[2] + out[3];
  if (!std::isfinite(out[0])) return set_error("objective is not finite"), MUFFIN_ENONFINITE;
  return MUFFIN_OK;
}

int muffin_step_monitored(muffin_ctx* c, int32_t n_iter, double out[6]) {
  if (!c || !out || n_iter < 1) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  if (!scope.ok) return set_error("stream ordering failed"), MUFFIN_EHIP;
  MF_TRY(ensure_graph(c));
  if (n_iter > 1) MF_TRY(replay(c, n_iter - 1));
  MF_TRY(snapshot_state(c));
  MF_TRY(replay(c, 1));
  c->iter += n_iter;
  return state_change(c, out);
}

int muffin_solve(muffin_ctx* c, int32_t max_iter, int32_t check_every, int32_t rule, double tol, double f_ref,
                 int32_t* iters_done, double* f_final) {
  if (!c || max_iter < 0 || check_every < 1 || !(tol >= 0) ||
      (rule != MUFFIN_STOP_OBJECTIVE && rule != MUFFIN_STOP_CHANGE))
    return set_error("bad arguments"), MUFFIN_EINVAL;
  int done = 0;
  double f = NAN, f_prev = NAN, o[4], nrm[6];
  auto rel = [](double d, double n) { return d == 0.0 ? 0.0 : d / n; };
  auto finish = [&](int rc) {
    if (iters_done) *iters_done = done;
    if (f_final) *f_final = f;
    return rc;
  };
  while (done < max_iter) {
    const int n = (max_iter - done < check_every) ? max_iter - done : check_every;
    bool stop = false;
    if (rule == MUFFIN_STOP_CHANGE) {
      const int rc = muffin_step_monitored(c, n, nrm);
      if (rc != MUFFIN_OK) return finish(rc);
      done += n;
      const double ch = std::fmax(rel(nrm[0], nrm[1]), std::fmax(rel(nrm[2], nrm[3]), rel(nrm[4], nrm[5])));
      if (!std::isfinite(ch)) return finish((set_error("iterates became non-finite"), MUFFIN_ENONFINITE));
      stop = ch <= tol;
    } else {
      MF_TRY(muffin_step(c, n));
      done += n;
    }
    if (rule == MUFFIN_STOP_OBJECTIVE || stop || done >= max_iter) {
      const int rc = muffin_objective(c, o);
      f = o[0];
      if (rc != MUFFIN_OK) return finish(rc);
    }
    if (rule == MUFFIN_STOP_OBJECTIVE) {
      if (std::isfinite(f_ref)) {
        stop = (f - f_ref) / std::fabs(f_ref) <= tol;
      } else {
        stop = std::isfinite(f_prev) && std::fabs(f - f_prev) <= tol * std::fabs(f);
      }
      f_prev = f;
    }
    if (stop) break;
  }
  if (done == 0) {
    const int rc = muffin_objective(c, o);
    f = o[0];
    if (rc != MUFFIN_OK) return finish(rc);
  }
  return finish(MUFFIN_OK);
}

int muffin_snr(muffin_ctx* c, const float* truth, int on_device, double* snr_db) {
  if (!c || !truth || !snr_db) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  return snr_of(c, 0, c->L, truth, on_device, snr_db);
}

// U = 0 (with the fused tail: current planes in U, carried adjoint sum zero, which is exact).
static int zero_dual(muffin_ctx* c) {
  MF_HIP(hipMemsetAsync(c->U, 0, sizeof(float) * c->ucube, c->st));
  if (c->fused) {
    MF_HIP(hipMemsetAsync(c->Acar, 0, sizeof(float) * c->cube, c->st));
    c->upar = 0;
    c->acar_ok = true;
  }
  MF_HIP(hipMemsetAsync(c->V, 0, sizeof(float) * c->cube, c->st));
  return MUFFIN_OK;
}

// U to or from the caller's dense [L][J+1][N][N] array.  With the fused tail's current planes
// in U2, its three planes of every channel are copied on their own.
static int u_out(muffin_ctx* c, float* dst, int on_device) {
  MF_TRY(planes_out(c, dst, c->U, (long long)c->L * c->np_u, on_device, c->us));
  if (c->fused && c->upar) {
    const long long np = c->npix;
    MF_TRY(copy_planes(dst + (long long)c->jf * np, c->np_u * np, c->U2, 3 * c->us, c->L, 3 * np,
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->st));
  }
  return MUFFIN_OK;
}
static int u_in(muffin_ctx* c, const float* src, int on_device) {
  MF_TRY(planes_in(c, c->U, src, (long long)c->L * c->np_u, on_device, c->us));
  if (c->fused) {
    c->upar = 0;
    c->acar_ok = false;  // recomputed before the next iteration
  }
  return MUFFIN_OK;
}

int muffin_info(muffin_ctx* c, double out[8]) {
  if (!c || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  const Seg& s = c->segs[0];
  out[0] = s.tau;
  out[1] = c->sigma;
  out[2] = c->rho;
  out[3] = s.beta;
  out[4] = s.K2;
  out[5] = c->Ws2;
  out[6] = s.delta;
  out[7] = (double)c->iter;
  return MUFFIN_OK;
}

int muffin_set_x(muffin_ctx* c, const float* x0, int on_device) {
  if (!c || !x0) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  MF_TRY(planes_in(c, c->X, x0, c->L, on_device));
  MF_TRY(launch_clamp_pos(c->X, c->cube, c->st));
  return zero_dual(c);
}

int muffin_get_x(muffin_ctx* c, float* x, int on_device) {
  if (!c || !x) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  return planes_out(c, x, c->X, c->L, on_device);
}
int muffin_get_u(muffin_ctx* c, float* u, int on_device) {
  if (!c || !u) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  return u_out(c, u, on_device);
}
int muffin_get_v(muffin_ctx* c, float* v, int on_device) {
  if (!c || !v) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  return planes_out(c, v, c->V, c->L, on_device);
}

int muffin_state_size(muffin_ctx* c, size_t* bytes) {
  if (!c || !bytes) return set_error("bad arguments"), MUFFIN_EINVAL;
  *bytes = sizeof(BlobHeader) + sizeof(float) * (size_t)c->npix * c->L * (c->np_u + 2);
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
  h.pad = blob_kind(c);
  h.mu_s = c->p.mu_s;
  h.mu_l = c->segs[0].mu_l;
  h.tau = c->segs[0].tau;
  h.sigma = c->sigma;
  h.rho = c->rho;
  h.iter = c->iter;
  std::memcpy(blob, &h, sizeof(h));
  float* f = (float*)((char*)blob + sizeof(h));
  StreamScope scope(c);
  const long long dense = c->npix * c->L;  // the blob holds X, U, V in the dense layout
  MF_TRY(planes_out(c, f, c->X, c->L, 0));
  MF_TRY(u_out(c, f + dense, 0));
  MF_TRY(planes_out(c, f + dense * (c->np_u + 1), c->V, c->L, 0));
  return MUFFIN_OK;
}

int muffin_set_state(muffin_ctx* c, const void* blob, size_t bytes) {
  size_t need = 0;
  MF_TRY(muffin_state_size(c, &need));
  if (!blob || bytes < need) return set_error("blob too small"), MUFFIN_ESTATE;
  BlobHeader h;
  std::memcpy(&h, blob, sizeof(h));
  if (h.magic != kMagic || h.N != c->N || h.L != c->L || h.J != c->J || h.gen != c->gen ||
      h.pc != c->p.penalize_coarse || h.pad != blob_kind(c) || h.mu_s != c->p.mu_s || h.mu_l != c->segs[0].mu_l || h.tau != c->segs[0].tau ||
      h.sigma != c->sigma || h.rho != c->rho)
    return set_error("checkpoint sizes or parameters differ from the context"), MUFFIN_ESTATE;
  const float* f = (const float*)((const char*)blob + sizeof(h));
  StreamScope scope(c);
  const long long dense = c->npix * c->L;
  MF_TRY(planes_in(c, c->X, f, c->L, 0));
  MF_TRY(u_in(c, f + dense, 0));
  MF_TRY(planes_in(c, c->V, f + dense * (c->np_u + 1), c->L, 0));
  c->iter = h.iter;
  return MUFFIN_OK;
}

int muffin_warm_input(muffin_ctx* c, float* out, int on_device) {
  if (!c || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  if (c->vis) return set_error("the warm start needs dirty images (image-plane context)"), MUFFIN_EINVAL;
  StreamScope scope(c);
  MF_TRY(cnn_warm_input(c->Y, c->cs, c->psf_lobe, c->cA, c->N, c->L, c->st));  // dense planes
  return copy_out(out, c->cA, (size_t)(c->npix * c->L), on_device, c->st);
}

int muffin_warm_start(muffin_ctx* c, muffin_cnn* net) {
  if (!c || !net) return set_error("bad arguments"), MUFFIN_EINVAL;
  if (c->vis) return set_error("the warm start needs dirty images (image-plane context)"), MUFFIN_EINVAL;
  if (c->N % 32) return set_error("warm start needs N to be a multiple of 32"), MUFFIN_EINVAL;
  StreamScope scope(c);
  MF_TRY(cnn_warm_input(c->Y, c->cs, c->psf_lobe, c->cA, c->N, c->L, c->st));  // dense planes
  // the network's stream runs after this stream's work so far, and this stream after the network's
  MF_TRY(cnn_predict_after(net, c->cA, c->cB, c->L, c->N, c->st));
  MF_TRY(planes_in(c, c->X, c->cB, c->L, 1));
  MF_TRY(launch_clamp_pos(c->X, c->cube, c->st));
  return zero_dual(c);
}

int muffin_apply_op(muffin_ctx* c, int op, const float* in, float* out) {
  if (!c || !in || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  StreamScope scope(c);
  // in and out are dense (planes np floats apart); the scratch planes use the library's slots
  const long long np = c->npix, cs = c->cs;
  const float inv_n2 = 1.f / ((float)c->N * c->N);
  const bool vis_op = op == MUFFIN_OP_PHI || op == MUFFIN_OP_PHI_ADJ;
  if (vis_op && !c->vis) return set_error("PHI operators need a visibility context"), MUFFIN_EINVAL;
  if ((op == MUFFIN_OP_H || op == MUFFIN_OP_HT) && c->vis)
    return set_error("H operators need an image-plane context"), MUFFIN_EINVAL;
  switch (op) {
    case MUFFIN_OP_PHI:
      // the residual with no data is Phi x; it also lands in out
      return enqueue_vis_forward(c, in, np, nullptr, 0.f, nullptr, nullptr, (float2*)out, false);
    case MUFFIN_OP_PHI_ADJ:
      // no bands: the residual is the operand itself
      MF_TRY(launch_vis_resid(nullptr, 0, c->L, c->K, (const float2*)in, 1.f, nullptr, c->vp, nullptr, nullptr,
                              nullptr, c->st));
      return launch_vis_adj(c->vp, c->K, c->L, c->vlt, c->vnt, c->vinvn, c->N, out, np, nullptr, 0, 0.f, c->st);
    case MUFFIN_OP_H:
    case MUFFIN_OP_HT:
      MF_TRY(launch_rows_r2c(in, np, c->S, c->L, c->g, c->tw, false, c->st));
      MF_TRY(launch_cols(c->S, c->L, c->g, c->tw, op == MUFFIN_OP_H ? COL_CPLX : COL_CPLX_CONJ, nullptr, c->Hhat_T,
                         inv_n2, nullptr, c->st));
      MF_TRY(launch_rows_c2r(c->S, c->L, c->g, c->tw, EPI_STORE, out, np, nullptr, nullptr, 0.f, nullptr, nullptr,
                             nullptr, nullptr, c->st));
      return MUFFIN_OK;
    case MUFFIN_OP_GRAD:
      // the epilogue reads b in the slots: the operand and result go through scratch planes
      MF_TRY(planes_in(c, c->cT, in, c->L, 1));
      MF_TRY(enqueue_gradient(c, c->cT, c->cA, nullptr, 0.f));
      return planes_out(c, out, c->cA, c->L, 1);
    case MUFFIN_OP_IUWT: {
      const long long ucs = (long long)c->np_u * np;
      if (c->uob)
        return enqueue_uob_analysis(c, UOB_STORE, in, np, 0, c->L, nullptr, 0, 0, out, ucs, np, 0.f, 1.f,
                                    (float)(1.0 / std::sqrt((double)kUobBases)), nullptr);
      const float* cur = in;
      float* bufs[2] = {c->cA, c->cB};
      for (int j = 0; j < c->J; ++j) {
        float* nxt = bufs[j & 1];
        const long long ccs = cur == in ? np : cs;
        MF_TRY(launch_atrous(SM_SMOOTH, c->N, c->L, j, pref(cur, ccs), PlaneRef{}, PlaneRef{}, pout(nxt, cs),
                             PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
        float* wj = out + (long long)j * np;
        if (c->gen == 2) {
          // w = c_j - H_j c_{j+1}: smooth c_{j+1} into the output plane, then subtract
          MF_TRY(launch_atrous(SM_SMOOTH, c->N, c->L, j, pref(nxt, cs), PlaneRef{}, PlaneRef{}, pout(c->cT, cs),
                               PlaneOut{}, 0.f, 1.f, nullptr, nullptr, c->st));
          MF_TRY(launch_pointwise(PT_SUB, c->N, c->L, pref(c->cT, cs), pref(cur, ccs), pout(wj, ucs), 0.f, 1.f,
                                  nullptr, nullptr, c->st));
        } else {
          MF_TRY(launch_pointwise(PT_SUB, c->N, c->L, pref(nxt, cs), pref(cur, ccs), pout(wj, ucs), 0.f, 1.f, nullptr,
                                  nullptr, c->st));
        }
        cur = nxt;
      }
      return launch_pointwise(PT_COPY, c->N, c->L, pref(cur, cs), PlaneRef{},
                              pout(out + (long long)c->J * np, ucs), 1.f, 1.f, nullptr, nullptr, c->st);
    }
    case MUFFIN_OP_IUWT_ADJ: {
      const float* a = nullptr;
      MF_TRY(enqueue_adjoint(c, in, np, (long long)c->np_u * np, 1.f, &a));
      return launch_pointwise(PT_COPY, c->N, c->L, pref(a, cs), PlaneRef{}, pout(out, np), 1.f, 1.f, nullptr,
                              nullptr, c->st);
    }
    case MUFFIN_OP_IUWT_SCHED: {
      // the iteration's own analysis launches (triples, pairs, the fused tail when the context uses
      // it) on zero dual planes with sigma mu_s = rho = 1: each dual plane becomes sat(w) = w
      const long long J1 = c->np_u, us = c->us;
      if (!c->Us) MF_TRY(dalloc(&c->Us, (long long)c->L * J1 * np));
      float *U2s = nullptr, *Acs = nullptr;
      if (c->fused) {
        MF_TRY(dalloc(&U2s, (long long)c->L * 3 * us));
        MF_TRY(dalloc(&Acs, c->cube));
        MF_HIP(hipMemsetAsync(U2s, 0, sizeof(float) * c->L * 3 * us, c->st));
      }
      MF_HIP(hipMemsetAsync(c->Us, 0, sizeof(float) * c->L * J1 * np, c->st));
      MF_TRY(planes_in(c, c->cT, in, c->L, 1));
      float *U0 = c->U, *U20 = c->U2, *Ac0 = c->Acar;
      const double sg = c->sigma, ms = c->p.mu_s, rh = c->rho;
      c->U = c->Us;
      c->U2 = U2s;
      c->Acar = Acs;
      c->sigma = 1.0;
      c->p.mu_s = 1.0;
      c->rho = 1.0;
      const int rc = enqueue_dual_update(c, c->cT, false, 0);
      c->U = U0;
      c->U2 = U20;
      c->Acar = Ac0;
      c->sigma = sg;
      c->p.mu_s = ms;
      c->rho = rh;
      int rc2 = rc;
      if (rc == MUFFIN_OK) {
        // planes below the fused tail's are in the dense scratch, the tail's three in its second buffer
        rc2 = copy_planes(out, J1 * np, c->Us, J1 * np, c->L, J1 * np, hipMemcpyDeviceToDevice, c->st);
        if (rc2 == MUFFIN_OK && c->fused)
          rc2 = copy_planes(out + (long long)c->jf * np, J1 * np, U2s, 3 * us, c->L, 3 * np, hipMemcpyDeviceToDevice,
                            c->st);
      }
      if (U2s || Acs) {
        (void)hipStreamSynchronize(c->st);
        if (U2s) (void)hipFree(U2s);
        if (Acs) (void)hipFree(Acs);
      }
      return rc2;
    }
    case MUFFIN_OP_DCT:
      return launch_dct(in, out, c->segs[0].WT, np, np, c->L, c->st);
    case MUFFIN_OP_IDCT:
      return launch_dct(in, out, c->segs[0].W, np, np, c->L, c->st);
    default:
      return set_error("unknown operator"), MUFFIN_EINVAL;
  }
}

}  // extern "C"
