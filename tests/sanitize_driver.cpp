// Host-side driver of the C ABI for the sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of lpt2_api.cpp): every
// validation and error path that runs without a device.  Prints one line per
// check and exits non-zero on the first unexpected status.
#include <cstdio>
#include <cstring>

#include "lpt2.h"

static int g_fail = 0;
#define EXPECT(cond, what)                          \
  do {                                              \
    if (!(cond)) {                                  \
      std::printf("FAIL %s\n", what);               \
      g_fail = 1;                                   \
    } else {                                        \
      std::printf("ok %s\n", what);                 \
    }                                               \
  } while (0)

static lpt2_status plan_with(void (*edit)(lpt2_config*), lpt2_plan_t* out) {
  lpt2_config c;
  lpt2_config_default(&c);
  if (edit) edit(&c);
  return lpt2_plan(&c, 1, nullptr, out);
}

int main() {
  // configurations refused on the host
  struct Case {
    const char* name;
    void (*edit)(lpt2_config*);
    lpt2_status want;
  } cases[] = {
      {"n=44", [](lpt2_config* c) { c->n = 44; }, LPT2_EUNSUPPORTED},
      {"n=1536", [](lpt2_config* c) { c->n = 1536; }, LPT2_EUNSUPPORTED},
      {"precision 7", [](lpt2_config* c) { c->precision = 7; }, LPT2_EUNSUPPORTED},
      {"box 0", [](lpt2_config* c) { c->box = 0.0; }, LPT2_EINVAL},
      {"fr0 0", [](lpt2_config* c) { c->gravity = LPT2_GRAV_FR_HS; c->fr0_abs = 0.0; }, LPT2_EINVAL},
      {"hs_n 2", [](lpt2_config* c) { c->gravity = LPT2_GRAV_FR_HS; c->hs_n = 2; }, LPT2_EUNSUPPORTED},
      {"gravity 9", [](lpt2_config* c) { c->gravity = 9; }, LPT2_EINVAL},
      {"factorisation 8", [](lpt2_config* c) { c->factorisation = 8; }, LPT2_EINVAL},
      {"nk 1", [](lpt2_config* c) { c->nk_growth = 1; }, LPT2_EINVAL},
      {"kmax < kmin", [](lpt2_config* c) { c->kmax = 1e-4; }, LPT2_EINVAL},
      {"a_init 0", [](lpt2_config* c) { c->a_init = 0.0; }, LPT2_EINVAL},
      {"steps 0", [](lpt2_config* c) { c->ode_steps = 0; }, LPT2_EINVAL},
      {"theta 180", [](lpt2_config* c) { c->factorisation = LPT2_D2_TRIANGLE; c->tri_theta_deg = 180.0; }, LPT2_EINVAL},
  };
  for (const Case& k : cases) {
    lpt2_plan_t p = reinterpret_cast<lpt2_plan_t>(0x1);
    const lpt2_status st = plan_with(k.edit, &p);
    EXPECT(st == k.want && p == nullptr && std::strlen(lpt2_last_error(nullptr)) > 0, k.name);
  }
  EXPECT(lpt2_plan(nullptr, 1, nullptr, nullptr) == LPT2_EINVAL, "plan out NULL");
  lpt2_config c;
  lpt2_config_default(&c);
  int zero = 0;
  lpt2_plan_t p = nullptr;
  EXPECT(lpt2_plan(&c, 1, &zero, &p) == LPT2_EINVAL && p == nullptr, "count 0");
  // a valid configuration: without a device the first allocation fails and
  // the partly built plan is released
  const lpt2_status st = lpt2_plan(&c, 1, nullptr, &p);
  std::printf("valid plan without a device: status %d (%s): %s\n", (int)st, lpt2_strerror(st), lpt2_last_error(nullptr));
  EXPECT(st == LPT2_OK || st == LPT2_ENOMEM || st == LPT2_EDEVICE, "valid plan status");
  if (st == LPT2_OK) lpt2_destroy(p);
  // every plan entry point refuses NULL
  double d = 0.0;
  int i = 0;
  long long ll = 0;
  EXPECT(lpt2_displace(nullptr, 1.0, nullptr, nullptr, nullptr, nullptr) == LPT2_EINVAL, "displace NULL");
  EXPECT(lpt2_displace_noalloc(nullptr, 1.0, nullptr, nullptr, nullptr, nullptr) == LPT2_EINVAL, "noalloc NULL");
  EXPECT(lpt2_backward(nullptr, 1.0, nullptr, nullptr, nullptr, nullptr, nullptr) == LPT2_EINVAL, "backward NULL");
  EXPECT(lpt2_source_spectrum(nullptr, 1.0, nullptr, 8, 0, &d, &d, &d, &d, nullptr) == LPT2_EINVAL, "spectrum NULL");
  EXPECT(lpt2_check_finite(nullptr, nullptr, 8, &ll, nullptr) == LPT2_EINVAL, "check_finite NULL");
  EXPECT(lpt2_growth_table(nullptr, 1.0, &d, &d, &d) == LPT2_EINVAL, "growth_table NULL");
  EXPECT(lpt2_auto_choice(nullptr, 0, 1.0, &i) == LPT2_EINVAL, "auto_choice NULL");
  EXPECT(lpt2_destroy(nullptr) == LPT2_OK, "destroy NULL");
  EXPECT(lpt2_realisations(nullptr) == 0, "realisations NULL");
  // status strings and the candidate table
  const lpt2_status all[] = {LPT2_OK, LPT2_EINVAL, LPT2_EUNSUPPORTED, LPT2_ENOMEM, LPT2_EDEVICE, LPT2_ESTATE};
  for (lpt2_status s : all) EXPECT(std::strlen(lpt2_strerror(s)) > 0, "strerror");
  EXPECT(std::strcmp(lpt2_strerror((lpt2_status)-99), "unknown status") == 0, "strerror unknown");
  const int nc = lpt2_factorisation_candidates();
  for (int k = 0; k < nc; ++k) {
    const char* name = nullptr;
    double r = 0.0, th = 0.0;
    int w = 0;
    EXPECT(lpt2_factorisation_candidate(k, &name, &r, &th, &w) == LPT2_OK && name && r > 0.0, "candidate");
  }
  EXPECT(lpt2_factorisation_candidate(nc, nullptr, nullptr, nullptr, nullptr) == LPT2_EINVAL, "candidate range");
  std::printf(g_fail ? "SANITIZE DRIVER FAILED\n" : "SANITIZE DRIVER OK\n");
  return g_fail;
}
