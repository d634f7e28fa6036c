// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library (device code is
// not built).  Every call here returns before any kernel launch: argument
// validation, the Hermiticity test, the diagonal-structure analysis of
// og_create / og_create_banded and the error paths that follow a failing
// device call.  Prints "ok" and returns 0 when every check holds.
#include <complex>
#include <cstdio>
#include <cstring>
#include <vector>

#include "opengrape.h"

typedef std::complex<double> C;

static int failures = 0;
#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "check failed, line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

// deterministic values in [-1, 1)
static double unit(unsigned long long& s) {
  s = s * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(s >> 11) / (double)(1ULL << 52) - 1.0;
}

static std::vector<C> hermitian(int d, unsigned long long seed) {
  std::vector<C> m((size_t)d * d);
  for (int i = 0; i < d; ++i)
    for (int j = i; j < d; ++j) {
      const C v(unit(seed), i == j ? 0.0 : unit(seed));
      m[(size_t)i * d + j] = v;
      m[(size_t)j * d + i] = std::conj(v);
    }
  return m;
}

int main() {
  for (int s = 0; s >= -8; --s) CHECK(og_status_string((og_status)s) != nullptr);
  og_options opt;
  og_default_options(&opt);
  CHECK(opt.prec == 0 && opt.gmode == 0 && opt.path == 0 && opt.n_sub == 1 && opt.ckpt_stride == 0 &&
        opt.validate == 1);

  og_ctx* ctx = nullptr;
  std::vector<C> eye(9);
  for (int i = 0; i < 3; ++i) eye[i * 4] = 1.0;
  CHECK(og_create(&ctx, 0, 0, 0, eye.data(), nullptr, nullptr, nullptr, nullptr) == OG_ERR_ARG);
  CHECK(og_create(&ctx, 3, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr) == OG_ERR_ARG);
  CHECK(og_create(nullptr, 3, 0, 0, eye.data(), nullptr, nullptr, nullptr, nullptr) == OG_ERR_ARG);
  std::vector<C> c1(9);
  const double neg = -1.0;
  CHECK(og_create(&ctx, 3, 0, 1, eye.data(), nullptr, c1.data(), &neg, nullptr) == OG_ERR_ARG);
  std::vector<C> bad = eye;
  bad[1] = 1.0;
  CHECK(og_create(&ctx, 3, 0, 0, bad.data(), nullptr, nullptr, nullptr, nullptr) == OG_ERR_NOT_HERMITIAN);
  CHECK(std::strstr(og_last_error(), "Hermitian") != nullptr);

  // a dense operator set with the banded path forced is a shape error
  const int d = 20;
  std::vector<C> H0 = hermitian(d, 1), Hk = hermitian(d, 2), cd = hermitian(d, 3);
  const double g1 = 0.5;
  og_options o2 = opt;
  o2.path = OG_PATH_BANDED;
  CHECK(og_create(&ctx, d, 1, 1, H0.data(), Hk.data(), cd.data(), &g1, &o2) == OG_ERR_SHAPE);
  o2 = opt;
  o2.n_sub = 0;
  CHECK(og_create(&ctx, 3, 0, 0, eye.data(), nullptr, nullptr, nullptr, &o2) == OG_ERR_ARG);

  // diagonal storage: argument errors, then a valid ladder structure (a
  // damped, driven resonator) whose creation ends at the first device call
  // when no GPU is present
  const int n = 12;
  const int offs[3] = {0, 1, -1};
  std::vector<C> h0d(3 * n), hkd(3 * n), cdd(3 * n);
  for (int i = 0; i < n; ++i) {
    h0d[i] = 0.3 * i;
    if (i + 1 < n) {
      hkd[n + i] = std::sqrt((double)(i + 1));  // (i, i + 1): a
      cdd[n + i] = std::sqrt((double)(i + 1));
    }
    if (i >= 1) hkd[2 * n + i] = std::sqrt((double)i);  // (i, i - 1): a^dag
  }
  CHECK(og_create_banded(&ctx, n, 0, 0, 0, offs, h0d.data(), nullptr, nullptr, nullptr, nullptr) == OG_ERR_ARG);
  CHECK(og_create_banded(&ctx, n, 0, 0, 2 * n, offs, h0d.data(), nullptr, nullptr, nullptr, nullptr) ==
        OG_ERR_ARG);
  const int rep[3] = {0, 1, 1};
  CHECK(og_create_banded(&ctx, n, 0, 0, 3, rep, h0d.data(), nullptr, nullptr, nullptr, nullptr) == OG_ERR_ARG);
  const int outside[3] = {0, 1, -n};
  CHECK(og_create_banded(&ctx, n, 0, 0, 3, outside, h0d.data(), nullptr, nullptr, nullptr, nullptr) ==
        OG_ERR_ARG);
  CHECK(og_create_banded(&ctx, n, 1, 0, 3, offs, h0d.data(), nullptr, nullptr, nullptr, nullptr) == OG_ERR_ARG);
  std::vector<C> badd = h0d;
  badd[n] = 1.0;
  CHECK(og_create_banded(&ctx, n, 0, 0, 3, offs, badd.data(), nullptr, nullptr, nullptr, nullptr) ==
        OG_ERR_NOT_HERMITIAN);
  og_ctx* ok = nullptr;
  const og_status st = og_create_banded(&ok, n, 1, 1, 3, offs, h0d.data(), hkd.data(), cdd.data(), &g1, nullptr);
  CHECK(st == OG_OK || st == OG_ERR_DEVICE);
  if (st == OG_OK) {
    CHECK(og_path_used(ok) == OG_PATH_BANDED);
    CHECK(og_destroy(ok) == OG_OK);
  } else {
    CHECK(ok == nullptr);
  }

  // NULL context everywhere
  CHECK(og_workspace_bytes(nullptr, 1, 1) == 0);
  CHECK(og_forward(nullptr, 1, 1, 0.1, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == OG_ERR_ARG);
  CHECK(og_cost(nullptr, nullptr, nullptr, nullptr) == OG_ERR_ARG);
  CHECK(og_adjoint(nullptr, nullptr, nullptr) == OG_ERR_ARG);
  CHECK(og_gradient(nullptr, nullptr, nullptr) == OG_ERR_ARG);
  CHECK(og_gradient_sum(nullptr, nullptr, 0, nullptr) == OG_ERR_ARG);
  CHECK(og_destroy(nullptr) == OG_OK);
  CHECK(og_set_adaptive(nullptr, 1e-6, 1e-8) == OG_ERR_ARG);
  CHECK(og_adaptive_stats(nullptr, nullptr) == OG_ERR_ARG);
  CHECK(og_set_resident(nullptr, 4) == OG_ERR_ARG);
  CHECK(og_generation(nullptr) == 0);
  CHECK(og_set_fused(nullptr, 1) == OG_ERR_ARG);
  CHECK(og_fused_used(nullptr) == 0);
  CHECK(og_set_penalty(nullptr, nullptr, 0.0) == OG_ERR_ARG);
  CHECK(og_evaluate_static(nullptr, 1, 1, 0.1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        OG_ERR_ARG);
  CHECK(og_server_create(nullptr, nullptr, 1) == OG_ERR_ARG);
  CHECK(og_profile(nullptr, 1) == OG_ERR_ARG);

  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
