// Host-side checks of libmuffin built with AddressSanitizer and UndefinedBehaviorSanitizer on its
// host code (test infrastructure; no GPU needed).  It runs the library's host logic: argument
// validation of every constructor (the visibility one included), error reporting, the Daubechies filter construction, the FFT
// twiddle tables and the Bluestein tables of the spectral step, and context creation without a
// usable device (the error path that tears a half-built context down).  Each table is checked
// against its definition, recomputed here in FP64.  Prints "host checks passed" and exits 0 when
// every check holds; any sanitizer report aborts the process.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "muffin.h"

namespace mf {
std::vector<float2> fft_twiddles(int N);
std::vector<float2> spectral_blu_table(int L);
int spectral_blu_m(int L);
bool spectral_has_fft(int L);
}  // namespace mf

static int failures = 0;
#define CHECK(cond)                                                     \
  do {                                                                  \
    if (!(cond)) {                                                      \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

static muffin_params base_params() {
  muffin_params p{};
  p.N = 64;
  p.L = 4;
  p.J = 2;
  p.iuwt_gen = 2;
  p.penalize_coarse = 1;
  p.mu_s = 0.1;
  p.mu_lambda = 0.1;
  p.sigma = 1.0;
  p.rho = 1.0;
  return p;
}

static void check_errors() {
  CHECK(std::string(muffin_strerror(MUFFIN_OK)) == "ok");
  for (int code = -6; code <= -1; ++code) CHECK(std::string(muffin_strerror(code)) != "unknown error");
  CHECK(std::string(muffin_strerror(-99)) == "unknown error");
}

static void check_validation() {
  std::vector<float> cube(64 * 64 * 4, 0.f);
  muffin_ctx* ctx = nullptr;
  CHECK(muffin_init(nullptr, nullptr, nullptr, nullptr, 0, nullptr) == MUFFIN_EINVAL);
  CHECK(muffin_init(&ctx, nullptr, cube.data(), cube.data(), 0, nullptr) == MUFFIN_EINVAL);
  struct Bad {
    void (*edit)(muffin_params&);
  };
  const Bad bad[] = {
      {[](muffin_params& p) { p.N = 100; }},       {[](muffin_params& p) { p.N = 2048; }},
      {[](muffin_params& p) { p.L = 0; }},         {[](muffin_params& p) { p.L = 513; }},
      {[](muffin_params& p) { p.J = 0; }},         {[](muffin_params& p) { p.J = 7; }},
      {[](muffin_params& p) { p.iuwt_gen = 3; }},  {[](muffin_params& p) { p.sigma = -1.0; }},
      {[](muffin_params& p) { p.mu_s = -1.0; }},   {[](muffin_params& p) { p.mu_lambda = NAN; }},
      {[](muffin_params& p) { p.flags = 1 << 20; }},
      {[](muffin_params& p) { p.flags = MUFFIN_FLAG_NO_FUSED_TAIL | MUFFIN_FLAG_FUSED_TAIL; }},
      {[](muffin_params& p) { p.flags = MUFFIN_FLAG_UOB_ALL_BASES | MUFFIN_FLAG_UOB_PER_BASIS; }},
      {[](muffin_params& p) { p.flags = MUFFIN_FLAG_SPECTRAL_DENSE | MUFFIN_FLAG_SPECTRAL_BLUESTEIN; }},
      {[](muffin_params& p) { p.prior = 2; }},
      {[](muffin_params& p) { p.prior = MUFFIN_PRIOR_UOB; p.N = 96; p.J = 6; }},
  };
  for (const Bad& b : bad) {
    muffin_params p = base_params();
    b.edit(p);
    ctx = reinterpret_cast<muffin_ctx*>(&p);  // must be reset to NULL on error
    CHECK(muffin_init(&ctx, &p, cube.data(), cube.data(), 0, nullptr) == MUFFIN_EINVAL);
    CHECK(ctx == nullptr);
    CHECK(std::string(muffin_last_error()).size() > 0);
  }
  // the batch constructor checks every cube
  muffin_params ps[2] = {base_params(), base_params()};
  ps[1].L = 0;
  const float* d[2] = {cube.data(), cube.data()};
  muffin_batch* batch = nullptr;
  CHECK(muffin_batch_init(&batch, 2, ps, d, d, 0, nullptr) == MUFFIN_EINVAL);
  CHECK(muffin_batch_init(&batch, 0, ps, d, d, 0, nullptr) == MUFFIN_EINVAL);
  CHECK(muffin_batch_init(nullptr, 2, ps, d, d, 0, nullptr) == MUFFIN_EINVAL);
  // the visibility constructor: its descriptor, geometry, wavelengths and baselines
  {
    std::vector<double> uvw(3 * 5, 1.0), lam(4, 1.0);
    std::vector<float> vis(2 * 5 * 4, 0.f);
    muffin_vis_desc d{};
    d.K = 5;
    d.cell = 1e-3;
    d.uvw = uvw.data();
    d.lambda = lam.data();
    muffin_params p = base_params();
    CHECK(muffin_init_vis(&ctx, &p, nullptr, vis.data(), 0, nullptr) == MUFFIN_EINVAL);
    CHECK(muffin_init_vis(&ctx, &p, &d, nullptr, 0, nullptr) == MUFFIN_EINVAL);
    struct BadVis {
      void (*edit)(muffin_params&, muffin_vis_desc&, std::vector<double>&, std::vector<double>&);
      int code;
    };
    const BadVis badv[] = {
        {[](muffin_params&, muffin_vis_desc& dd, std::vector<double>&, std::vector<double>&) { dd.K = 0; },
         MUFFIN_EINVAL},
        {[](muffin_params&, muffin_vis_desc& dd, std::vector<double>&, std::vector<double>&) { dd.cell = 0.03; },
         MUFFIN_EINVAL},  // the corner pixel leaves the unit disc
        {[](muffin_params&, muffin_vis_desc& dd, std::vector<double>&, std::vector<double>&) { dd.cell = NAN; },
         MUFFIN_EINVAL},
        {[](muffin_params& pp, muffin_vis_desc&, std::vector<double>&, std::vector<double>&) { pp.N = 12; },
         MUFFIN_EINVAL},  // not a multiple of 8
        {[](muffin_params&, muffin_vis_desc&, std::vector<double>&, std::vector<double>& ll) { ll[2] = -1.0; },
         MUFFIN_EINVAL},
        {[](muffin_params&, muffin_vis_desc&, std::vector<double>& uu, std::vector<double>&) { uu[7] = INFINITY; },
         MUFFIN_ENONFINITE},
        {[](muffin_params&, muffin_vis_desc& dd, std::vector<double>&, std::vector<double>&) { dd.power_iters = -1; },
         MUFFIN_EINVAL},
    };
    for (const BadVis& b : badv) {
      muffin_params pp = base_params();
      muffin_vis_desc dd = d;
      std::vector<double> uu = uvw, ll = lam;
      b.edit(pp, dd, uu, ll);
      dd.uvw = uu.data();
      dd.lambda = ll.data();
      ctx = reinterpret_cast<muffin_ctx*>(&pp);  // must be reset to NULL on error
      CHECK(muffin_init_vis(&ctx, &pp, &dd, vis.data(), 0, nullptr) == b.code);
      CHECK(ctx == nullptr);
    }
    float cw[4] = {1.f, 0.f, 1.f, 1.f};  // a channel weight must be > 0
    p.chan_weight = cw;
    CHECK(muffin_init_vis(&ctx, &p, &d, vis.data(), 0, nullptr) == MUFFIN_EINVAL);
    CHECK(muffin_vis_residual(nullptr, vis.data(), 0) == MUFFIN_EINVAL);
  }
  // launch tiles: rows must divide N, class groups a power of two up to min(2^j, 8), known families
  CHECK(muffin_set_band_tiles(64, 2, MUFFIN_FAMILY_PAIR_ANALYSIS, 24, 1) == MUFFIN_EINVAL);
  CHECK(muffin_set_band_tiles(64, 2, MUFFIN_FAMILY_PAIR_ANALYSIS, 16, 8) == MUFFIN_EINVAL);
  CHECK(muffin_set_band_tiles(64, 4, MUFFIN_FAMILY_TRIPLE_ADJOINT, 16, 16) == MUFFIN_EINVAL);
  CHECK(muffin_set_band_tiles(64, 3, MUFFIN_FAMILY_FUSED_PAIR, 16, 3) == MUFFIN_EINVAL);
  CHECK(muffin_set_band_tiles(64, 3, 4, 16, 1) == MUFFIN_EINVAL);
  CHECK(muffin_set_band_tiles(64, 3, 12, 16, 1) == MUFFIN_EINVAL);
  CHECK(muffin_set_band_tiles(0, 3, MUFFIN_FAMILY_ANALYSIS, 0, 0) == MUFFIN_EINVAL);
  CHECK(muffin_set_band_tiles(64, -1, MUFFIN_FAMILY_ANALYSIS, 0, 0) == MUFFIN_EINVAL);
  CHECK(muffin_set_band_tiles(64, 3, MUFFIN_FAMILY_FUSED_PAIR, 32, 8) == MUFFIN_OK);
  CHECK(muffin_set_band_tiles(64, 3, MUFFIN_FAMILY_FUSED_PAIR, 0, 0) == MUFFIN_OK);
  // calls on NULL handles
  double out[8];
  CHECK(muffin_step(nullptr, 1) == MUFFIN_EINVAL);
  CHECK(muffin_objective(nullptr, out) == MUFFIN_EINVAL);
  CHECK(muffin_info(nullptr, out) == MUFFIN_EINVAL);
  CHECK(muffin_batch_step(nullptr, 1) == MUFFIN_EINVAL);
  muffin_free(nullptr);
  muffin_batch_free(nullptr);
}

// A valid context on a machine without a usable device fails with a HIP error and leaves nothing
// behind; on a machine with one it is created and freed.
static void check_context_lifecycle() {
  std::vector<float> dirty(64 * 64 * 4, 0.f), psf(64 * 64 * 4, 0.f);
  for (int l = 0; l < 4; ++l) psf[(size_t)l * 64 * 64 + 32 * 64 + 32] = 1.f;
  muffin_params p = base_params();
  muffin_ctx* ctx = nullptr;
  const int rc = muffin_init(&ctx, &p, dirty.data(), psf.data(), 0, nullptr);
  if (rc == MUFFIN_OK) {
    CHECK(ctx != nullptr);
    CHECK(muffin_step(ctx, 2) == MUFFIN_OK);
    muffin_free(ctx);
  } else {
    CHECK(rc == MUFFIN_EHIP || rc == MUFFIN_ENOMEM);
    CHECK(ctx == nullptr);
  }
}

static void check_filters() {
  double h[16];
  for (int n = 1; n <= 8; ++n) {
    CHECK(muffin_uob_filter(n, h, 16) == MUFFIN_OK);
    double sum = 0, norm = 0;
    for (int k = 0; k < 2 * n; ++k) sum += h[k], norm += h[k] * h[k];
    CHECK(std::fabs(sum - std::sqrt(2.0)) < 1e-12);
    CHECK(std::fabs(norm - 1.0) < 1e-12);
    for (int s = 1; s < n; ++s) {  // orthogonal to its even shifts
      double dot = 0;
      for (int k = 0; k + 2 * s < 2 * n; ++k) dot += h[k] * h[k + 2 * s];
      CHECK(std::fabs(dot) < 1e-12);
    }
  }
  CHECK(muffin_uob_filter(0, h, 16) == MUFFIN_EINVAL);
  CHECK(muffin_uob_filter(9, h, 18) == MUFFIN_EINVAL);
  CHECK(muffin_uob_filter(4, h, 7) == MUFFIN_EINVAL);
  CHECK(muffin_uob_filter(4, nullptr, 8) == MUFFIN_EINVAL);
}

static void check_twiddles() {
  for (int N : {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024}) {
    const std::vector<float2> w = mf::fft_twiddles(N);
    CHECK((int)w.size() == N);
    for (int m = 0; m < N; ++m) {
      const double th = -2.0 * M_PI * m / N;
      CHECK(std::fabs(w[m].x - std::cos(th)) < 1e-6 && std::fabs(w[m].y - std::sin(th)) < 1e-6);
    }
  }
}

// The Bluestein table of L: twiddles of M, FFT_M of the chirp conj(c_j) (|j| < L at j mod M) and
// the chirp c_n = exp(-i pi n^2 / L); and the identity it serves, DFT_L(z) = c . IFFT(FFT(z c) B),
// evaluated in FP64 from the FP32 table at a few outputs.
static void check_bluestein() {
  using cd = std::complex<double>;
  int tested = 0;
  for (int L = 16; L <= 512; ++L) {
    const int M = mf::spectral_blu_m(L);
    if (mf::spectral_has_fft(L)) {
      CHECK(M == 0);
      continue;
    }
    CHECK(M >= 2 * L - 1);
    if (L % 37 != 0 && L != 17 && L != 511) continue;  // the full check on a spread of lengths
    ++tested;
    const std::vector<float2> t = mf::spectral_blu_table(L);
    CHECK((int)t.size() == 2 * M + L);
    std::vector<cd> B(M), c(L);
    for (int k = 0; k < M; ++k) B[k] = cd(t[M + k].x, t[M + k].y);
    for (int n = 0; n < L; ++n) {
      c[n] = cd(t[2 * M + n].x, t[2 * M + n].y);
      CHECK(std::abs(c[n] - std::polar(1.0, -M_PI * (double)((long long)n * n % (2 * L)) / L)) < 1e-6);
    }
    // z_n = a fixed sequence; direct DFT against the convolution form (plain O(M^2) DFTs in FP64)
    std::vector<cd> z(L), a(M, 0.0), A(M), y(M);
    for (int n = 0; n < L; ++n) z[n] = cd(std::sin(0.3 * n + 1.0), std::cos(0.17 * n * n));
    for (int n = 0; n < L; ++n) a[n] = z[n] * c[n];
    for (int k = 0; k < M; ++k) {
      cd s = 0;
      for (int n = 0; n < M; ++n) s += a[n] * std::polar(1.0, -2.0 * M_PI * (double)((long long)n * k % M) / M);
      A[k] = s * B[k];
    }
    for (int k : {0, 1, L / 2, L - 1}) {
      cd s = 0;
      for (int m = 0; m < M; ++m) s += A[m] * std::polar(1.0, 2.0 * M_PI * (double)((long long)m * k % M) / M);
      const cd got = c[k] * s / (double)M;
      cd ref = 0;
      double scale = 0;
      for (int n = 0; n < L; ++n) {
        ref += z[n] * std::polar(1.0, -2.0 * M_PI * (double)((long long)n * k % L) / L);
        scale += std::abs(z[n]);
      }
      CHECK(std::abs(got - ref) < 1e-5 * scale);
    }
  }
  CHECK(tested >= 10);
}

int main() {
  check_errors();
  check_validation();
  check_filters();
  check_twiddles();
  check_bluestein();
  check_context_lifecycle();
  if (failures) {
    std::fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
