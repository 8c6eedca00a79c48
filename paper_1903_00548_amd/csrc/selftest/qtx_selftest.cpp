// Self-test of the C ABI's host logic, for builds with the host code under
// AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged).
// It drives every entry point through its argument checks, staging,
// workspace planning and launch sequences on small synthetic problems and
// checks what must hold whatever the numbers: status codes, outputs
// finite, equal results from entry points that promise them.
//
//   qtx_selftest          host-only part (no device needed)
//   qtx_selftest --gpu    everything, on device 0
//
// Prints "selftest: ok" and returns 0, or names the first failed check and
// returns 1.  Sanitizer reports abort the run on their own.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <vector>

#include "qtx.h"

namespace {

int g_fail = 0;

#define CHECK(cond)                                                                   \
  do {                                                                                \
    if (!(cond)) {                                                                    \
      std::fprintf(stderr, "selftest: check failed at line %d: %s\n", __LINE__, #cond); \
      g_fail = 1;                                                                     \
      return;                                                                         \
    }                                                                                 \
  } while (0)

// deterministic uniform numbers in [-1, 1)
struct Lcg {
  unsigned long long s;
  double next() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
};

using cd = std::complex<double>;

// A lead of block size m: Hermitian H00, small random H01 and S01, S00 = I
// plus a small Hermitian part.
struct Lead {
  int m;
  std::vector<qtx_c128> H00, H01, S00, S01;
};

Lead make_lead(int m, unsigned long long seed) {
  Lcg r{seed};
  Lead L{m, std::vector<qtx_c128>(m * m), std::vector<qtx_c128>(m * m), std::vector<qtx_c128>(m * m),
         std::vector<qtx_c128>(m * m)};
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j) {
      const double a = 2.0 * r.next(), b = i == j ? 0.0 : r.next();
      L.H00[i * m + j] = {a, b};
      L.H00[j * m + i] = {a, -b};
      const double s = i == j ? 1.0 : 0.02 * r.next(), t = i == j ? 0.0 : 0.02 * r.next();
      L.S00[i * m + j] = {s, t};
      L.S00[j * m + i] = {s, -t};
    }
  const double sc = 1.0 / m;
  for (int k = 0; k < m * m; ++k) {
    L.H01[k] = {sc * r.next(), sc * r.next()};
    L.S01[k] = {0.01 * sc * r.next(), 0.01 * sc * r.next()};
  }
  return L;
}

bool finite(const double* x, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(x[k])) return false;
  return true;
}

// a problem: both leads from one seed (right lead shifted by V), the device
// copying the left lead, a linear potential
bool fill(qtx_ctx* c, int N, int m, unsigned long long seed, double VR) {
  const Lead L = make_lead(m, seed);
  if (qtx_set_lead(c, QTX_LEFT, m, L.H00.data(), L.H01.data(), L.S00.data(), L.S01.data(), 0.0) != QTX_OK) return false;
  if (qtx_set_lead(c, QTX_RIGHT, m, L.H00.data(), L.H01.data(), L.S00.data(), L.S01.data(), VR) != QTX_OK) return false;
  if (qtx_set_device(c, N, m, nullptr, nullptr, nullptr, nullptr) != QTX_OK) return false;
  std::vector<double> V(N);
  for (int i = 0; i < N; ++i) V[i] = N > 1 ? VR * i / (N - 1) : 0.0;
  return qtx_set_potential(c, V.data(), QTX_POT_LINEAR_FE) == QTX_OK;
}

void host_only() {
  char msg[512];
  CHECK(qtx_check_layouts(msg, sizeof msg) == 0);
  CHECK(std::strncmp(msg, "ok:", 3) == 0);
  CHECK(qtx_check_layouts(nullptr, 0) == 0);
  CHECK(qtx_version() != nullptr && std::strlen(qtx_version()) > 0);
  qtx_ctx* c = nullptr;
  CHECK(qtx_create(-1, &c) != QTX_OK && c == nullptr);
  CHECK(qtx_create(0, nullptr) == QTX_EINVAL);
  CHECK(qtx_solve(nullptr, nullptr, 0, 0.0, QTX_FP64, nullptr, nullptr, nullptr) == QTX_EINVAL);
  CHECK(qtx_set_option(nullptr, "refine_tol", 1e-12) == QTX_EINVAL);
  CHECK(qtx_last_error(nullptr) != nullptr);
  qtx_destroy(nullptr);
  // the host charge helper: two energies, two slabs
  const double ldos[8] = {1, 2, 3, 4, 5, 6, 7, 8}, w[2] = {0.5, 0.5}, E[2] = {-0.1, 0.1};
  double q[2] = {0, 0};
  CHECK(qtx_charge(ldos, w, 2, 2, E, 0.0, 0.0, 0.025, q) == QTX_OK && finite(q, 2));
  CHECK(qtx_charge(ldos, w, 2, 2, E, 0.0, 0.0, -1.0, q) == QTX_EINVAL);
}

void on_device() {
  qtx_ctx* c = nullptr;
  CHECK(qtx_create(0, &c) == QTX_OK && c != nullptr);
  const int N = 7, m = 10, nE = 40;
  // calls out of order and bad arguments
  std::vector<double> E(nE), T(nE), T2(nE), ld(nE * 2 * N), ld2(nE * 2 * N);
  std::vector<qtx_info> info(nE);
  for (int k = 0; k < nE; ++k) E[k] = -1.2 + 2.4 * k / (nE - 1);
  CHECK(qtx_solve(c, E.data(), nE, 1e-6, QTX_FP64, T.data(), ld.data(), info.data()) == QTX_ESTATE);
  CHECK(fill(c, N, m, 11, -0.05));
  CHECK(qtx_solve(c, E.data(), nE, -1.0, QTX_FP64, T.data(), nullptr, nullptr) == QTX_EINVAL);
  CHECK(qtx_solve(c, nullptr, nE, 1e-6, QTX_FP64, T.data(), nullptr, nullptr) == QTX_EINVAL);
  CHECK(qtx_set_option(c, "no_such_option", 1.0) == QTX_EINVAL);
  CHECK(qtx_set_option(c, "refine_tol", -1.0) == QTX_EINVAL);
  // host-buffer solves: FP64 twice bit for bit, mixed within 1e-8
  CHECK(qtx_solve(c, E.data(), nE, 1e-6, QTX_FP64, T.data(), ld.data(), info.data()) == QTX_OK);
  CHECK(qtx_solve(c, E.data(), nE, 1e-6, QTX_FP64, T2.data(), ld2.data(), nullptr) == QTX_OK);
  CHECK(T == T2 && ld == ld2 && finite(T.data(), nE) && finite(ld.data(), ld.size()));
  CHECK(qtx_solve(c, E.data(), nE, 1e-6, QTX_MIXED, T2.data(), ld2.data(), info.data()) != QTX_EINVAL);
  for (int k = 0; k < nE; ++k) CHECK(std::fabs(T2[k] - T[k]) <= 1e-8);
  // device buffers: solve_device and the no-allocation variant
  double *Ed, *Td, *Ld;
  CHECK(hipMalloc(&Ed, nE * sizeof(double)) == hipSuccess);
  CHECK(hipMalloc(&Td, nE * sizeof(double)) == hipSuccess);
  CHECK(hipMalloc(&Ld, ld.size() * sizeof(double)) == hipSuccess);
  CHECK(hipMemcpy(Ed, E.data(), nE * sizeof(double), hipMemcpyHostToDevice) == hipSuccess);
  for (int mode = 0; mode < 2; ++mode) {
    const qtx_status s = mode == 0 ? qtx_solve_device(c, Ed, nE, 1e-6, QTX_FP64, Td, Ld, nullptr)
                                   : qtx_solve_device_noalloc(c, Ed, nE, 1e-6, QTX_FP64, Td, Ld, nullptr);
    CHECK(s == QTX_OK);
    CHECK(hipDeviceSynchronize() == hipSuccess);
    CHECK(hipMemcpy(T2.data(), Td, nE * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess);
    CHECK(hipMemcpy(ld2.data(), Ld, ld.size() * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess);
    CHECK(T2 == T && ld2 == ld);
  }
  // self-energies, charge, bands, density-matrix blocks
  std::vector<qtx_c128> sig(nE * 2 * m * m), wf(nE * 2 * m * m);
  std::vector<double> sg(nE * 2 * m);
  std::vector<int> it(nE);
  CHECK(qtx_self_energy(c, E.data(), nE, 1e-6, sig.data(), wf.data(), sg.data(), it.data()) == QTX_OK);
  for (int k = 0; k < nE; ++k) CHECK(it[k] > 0);
  std::vector<double> w(nE, 2.4 / (nE - 1)), q(N);
  CHECK(qtx_charge(ld.data(), w.data(), nE, N, E.data(), 0.1, -0.1, 0.025, q.data()) == QTX_OK && finite(q.data(), N));
  const double kk[3] = {0.0, 1.0, 3.14159};
  std::vector<double> Eb(3 * m);
  CHECK(qtx_bands(c, QTX_LEFT, kk, 3, Eb.data()) == QTX_OK && finite(Eb.data(), Eb.size()));
  std::vector<qtx_c128> rd(N * m * m), ro((N - 1) * m * m);
  std::vector<double> wl(nE, 0.3), wr(nE, 0.7);
  CHECK(qtx_density_matrix(c, E.data(), wl.data(), wr.data(), nE, 1e-6, rd.data(), ro.data(), nullptr, nullptr,
                           nullptr) == QTX_OK);
  // autotune on a small sample, then the same results from the tuned shape
  qtx_tune best, cand[QTX_TUNE_MAX_CANDIDATES];
  double tms[QTX_TUNE_MAX_CANDIDATES];
  int nc = 0;
  CHECK(qtx_autotune(c, E.data(), 8, 1e-6, QTX_FP64, &best, cand, tms, &nc) == QTX_OK && nc >= 1);
  CHECK(qtx_solve(c, E.data(), nE, 1e-6, QTX_FP64, T2.data(), nullptr, nullptr) == QTX_OK);
  for (int k = 0; k < nE; ++k) CHECK(std::fabs(T2[k] - T[k]) <= 1e-9);
  // batch: three problems of two block sizes, equal to the solo solves
  qtx_ctx* p[3] = {nullptr, nullptr, nullptr};
  const int pN[3] = {5, 9, 3}, pm[3] = {10, 20, 10}, pn[3] = {17, 9, 30};
  std::vector<std::vector<double>> pE(3), pT(3), pL(3);
  for (int j = 0; j < 3; ++j) {
    CHECK(qtx_problem_create(c, &p[j]) == QTX_OK);
    CHECK(fill(p[j], pN[j], pm[j], 100 + j, -0.02 * j));
    pE[j].resize(pn[j]);
    for (int k = 0; k < pn[j]; ++k) pE[j][k] = -1.0 + 1.9 * k / pn[j];
    pT[j].resize(pn[j]);
    pL[j].resize(pn[j] * 2 * pN[j]);
  }
  const double* Eptr[3] = {pE[0].data(), pE[1].data(), pE[2].data()};
  double* Tptr[3] = {pT[0].data(), pT[1].data(), pT[2].data()};
  double* Lptr[3] = {pL[0].data(), pL[1].data(), pL[2].data()};
  for (int rep = 0; rep < 2; ++rep) {             // the second call replays the captured graph
    CHECK(qtx_solve_batch(c, 3, p, Eptr, pn, 1e-6, QTX_FP64, Tptr, Lptr) == QTX_OK);
    for (int j = 0; j < 3; ++j) {
      std::vector<double> Ts(pn[j]), Ls(pL[j].size());
      CHECK(qtx_solve(p[j], pE[j].data(), pn[j], 1e-6, QTX_FP64, Ts.data(), Ls.data(), nullptr) == QTX_OK);
      CHECK(Ts == pT[j] && Ls == pL[j]);
    }
  }
  long long hits = 0, misses = 0, slots = 0;
  CHECK(qtx_sigma_cache_stats(c, &hits, &misses, &slots) == QTX_OK);
  // mode-space self-energies at eta = 0
  CHECK(qtx_set_option(c, "self_energy_method", 1) == QTX_OK);
  CHECK(qtx_solve(c, E.data(), nE, 0.0, QTX_FP64, T2.data(), nullptr, nullptr) != QTX_EINVAL);
  CHECK(finite(T2.data(), nE));
  CHECK(qtx_solve(c, E.data(), nE, 1e-6, QTX_FP64, T2.data(), nullptr, nullptr) == QTX_EINVAL);
  CHECK(qtx_set_option(c, "self_energy_method", 0) == QTX_OK);
  double dms = 0, sms = 0;
  int nl = 0;
  CHECK(qtx_kernel_times(c, 1, &dms, &sms, &nl) == QTX_OK);
  CHECK(qtx_solve(c, E.data(), nE, 1e-6, QTX_FP64, T2.data(), nullptr, nullptr) == QTX_OK);
  CHECK(qtx_kernel_times(c, 0, &dms, &sms, &nl) == QTX_OK && nl >= 1);
  for (int j = 0; j < 3; ++j) qtx_destroy(p[j]);
  CHECK(hipFree(Ed) == hipSuccess && hipFree(Td) == hipSuccess && hipFree(Ld) == hipSuccess);
  qtx_destroy(c);
}

}  // namespace

int main(int argc, char** argv) {
  const bool gpu = argc > 1 && std::strcmp(argv[1], "--gpu") == 0;
  host_only();
  if (!g_fail && gpu) on_device();
  if (g_fail) return 1;
  std::printf("selftest: ok (%s)\n", gpu ? "host and device" : "host only");
  return 0;
}
