// Host-side paths of the C ABI that run without a GPU, for a build of the
// library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
// configuration defaults, the rate table in every mode, every argument check
// of lbm_create, NULL handling, and the clean-up of a context whose device
// set-up fails.  Exit status = number of unexpected results.
#include <cmath>
#include <cstdio>

#include "lbm.h"

static int bad = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("unexpected: %s (last error: %s)\n", what, lbm_last_error(nullptr));
    ++bad;
  }
}

static lbm_config valid() {
  lbm_config c;
  lbm_config_default(&c);
  c.nx = 70;
  c.ny = 9;
  c.nz = 5;
  c.nu = 0.01;
  return c;
}

int main() {
  double w[LBM_Q];
  lbm_config c = valid();
  expect(lbm_omega_table(&c, w) == LBM_OK && std::fabs(w[4] - 1.0 / (3.0 * 0.01 + 0.5)) < 1e-15, "paper rates");
  c.omega_mode = LBM_OMEGA_ORDER_SCALED;
  expect(lbm_omega_table(&c, w) == LBM_OK && w[26] > 0.0 && w[26] < 2.0, "order-scaled rates");
  c.omega_mode = LBM_OMEGA_EXPLICIT;
  for (int j = 0; j < LBM_Q; ++j) c.omega[j] = 0.5 + 0.05 * j;
  expect(lbm_omega_table(&c, w) == LBM_OK && w[20] == c.omega[20], "explicit rates");
  c.omega[5] = 2.5;
  expect(lbm_omega_table(&c, w) == LBM_EINVAL, "explicit rate out of (0, 2)");
  expect(lbm_omega_table(nullptr, w) == LBM_EINVAL && lbm_omega_table(&c, nullptr) == LBM_EINVAL, "NULL table args");

  lbm_ctx* ctx = nullptr;
  struct Case { const char* what; void (*bend)(lbm_config&); };
  const Case cases[] = {
      {"zero grid", [](lbm_config& k) { k.ny = 0; }},
      {"2^31 nodes", [](lbm_config& k) { k.nx = 2048; k.ny = 1024; k.nz = 1024; }},
      {"unknown storage", [](lbm_config& k) { k.storage = (lbm_storage)9; }},
      {"walls_y 2", [](lbm_config& k) { k.walls_y = 2; }},
      {"walls_x 3", [](lbm_config& k) { k.walls_x = 3; }},
      {"NaN lid", [](lbm_config& k) { k.walls_y = 1; k.lid_velocity[1] = NAN; }},
      {"lid without walls", [](lbm_config& k) { k.lid_velocity[0] = 0.05; }},
      {"symmetry plane without wall", [](lbm_config& k) { k.sym_top = 1; }},
      {"negative LES constant", [](lbm_config& k) { k.les_cs = -0.1; }},
      {"LES without A+", [](lbm_config& k) { k.les_cs = 0.1; k.les_aplus = 0.0; }},
      {"unknown attractor", [](lbm_config& k) { k.attractor = (lbm_attractor)7; }},
      {"infinite force", [](lbm_config& k) { k.force[2] = INFINITY; }},
      {"negative viscosity", [](lbm_config& k) { k.nu = -0.01; }},
      {"bulk rate 2", [](lbm_config& k) { k.omega_bulk = 2.0; }},
  };
  for (const Case& k : cases) {
    lbm_config b = valid();
    k.bend(b);
    ctx = reinterpret_cast<lbm_ctx*>(&b);  // must be reset to NULL
    expect(lbm_create(&b, &ctx) == LBM_EINVAL && ctx == nullptr && lbm_last_error(nullptr)[0] != '\0', k.what);
  }
  expect(lbm_create(nullptr, &ctx) == LBM_EINVAL, "NULL config");
  expect(lbm_create(&c, nullptr) == LBM_EINVAL, "NULL out");
  // a valid configuration: without a GPU the device set-up fails after the
  // host context exists; it must be reported and released
  lbm_config v = valid();
  const int rc = lbm_create(&v, &ctx);
  if (rc == LBM_OK) {
    lbm_destroy(ctx);  // a GPU is visible after all: nothing more to check here
  } else {
    expect(rc == LBM_EHIP || rc == LBM_ENOMEM, "device set-up failure code");
    expect(ctx == nullptr, "no context after a failed create");
  }
  lbm_destroy(nullptr);
  std::printf("%d unexpected results\n", bad);
  return bad;
}
