// TEST INFRASTRUCTURE: exercises the host-side logic of the C ABI (argument
// validation, parameter resolution, workspace layout and the failure paths
// of lb_create that return before any device call) so that the runtime can
// be built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
// and run without a GPU. Exit status 0 when every call returned what the
// header promises.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lb.h"

static int fails = 0;
#define EXPECT(cond)                                     \
  do {                                                   \
    if (!(cond)) {                                       \
      std::printf("FAILED line %d: %s\n", __LINE__, #cond); \
      ++fails;                                           \
    }                                                    \
  } while (0)

static lb_channel chan(int nx, int ny) {
  lb_channel c;
  std::memset(&c, 0, sizeof c);
  c.nx = nx;
  c.ny = ny;
  c.force = 1e-6;
  c.tau_lb = 1.0;
  c.G = 1e-4;
  c.tau0 = 1e4;
  c.gamma_c = 0.1;
  c.t_startup = 1000;
  c.nn_pressure = 1;
  c.top_wall = LB_WALL_HALFWAY;
  return c;
}

int main() {
  lb_options o64 = {LB_FP64, 1000, 0, 0.0, 0, 0}, o32 = {LB_FP32_SHIFTED, 1000, 16, 1e-9, 0, 0};
  // every width class, ragged widths, one- and two-row channels, the drives
  std::vector<lb_channel> cs;
  const int shapes[][2] = {{1, 16}, {2, 9}, {8, 64}, {64, 7}, {100, 37}, {128, 9}, {256, 3}, {512, 11},
                           {768, 2}, {3, 1}, {4096, 1024}};
  for (auto &s : shapes) cs.push_back(chan(s[0], s[1]));
  lb_channel zh = chan(64, 9);
  zh.top_wall = LB_WALL_ZOU_HE;
  zh.wall_velocity = 0.02;
  zh.nn_pressure = 0;
  cs.push_back(zh);
  lb_channel pg = chan(100, 13);
  pg.force = 0;
  pg.pressure_gradient = 2e-6;
  pg.nn_pressure = 0;
  cs.push_back(pg);
  lb_channel st = chan(16, 40);
  st.visc_split = 0.5;
  st.nn_pressure = 0;
  st.eps = 0.07;
  cs.push_back(st);
  size_t b64 = 0, b32 = 0, bve = 0;
  EXPECT(lb_workspace_bytes(cs.data(), (int)cs.size(), &o64, &b64) == LB_OK && b64 > 0);
  EXPECT(lb_workspace_bytes(cs.data(), (int)cs.size(), &o32, &b32) == LB_OK && b32 > 0 && b32 < b64);
  lb_options ove = o32;
  ove.viscoelastic = 1;
  EXPECT(lb_workspace_bytes(cs.data(), (int)cs.size(), &ove, &bve) == LB_OK && bve > b32);
  lb_options osf = o64;
  osf.stress_force = 1;
  std::vector<lb_channel> sf = {chan(64, 8), chan(67, 5)};
  for (auto &c : sf) c.nn_pressure = 0;
  size_t bsf = 0;
  EXPECT(lb_workspace_bytes(sf.data(), 2, &osf, &bsf) == LB_OK && bsf > 0);
  // rejected inputs
  size_t b = 0;
  auto bad = [&](lb_channel c, const lb_options &o) { return lb_workspace_bytes(&c, 1, &o, &b) == LB_EINVAL; };
  lb_channel c = chan(8, 8);
  c.tau_lb = 0.5;
  EXPECT(bad(c, o64));
  c = chan(8, 8);
  c.top_wall = 3;
  EXPECT(bad(c, o64));
  c = chan(8, 1);
  c.top_wall = LB_WALL_ZOU_HE;
  EXPECT(bad(c, o64));
  c = chan(8, 8);
  c.nn_pressure = 2;
  EXPECT(bad(c, o64));
  c = chan(8, 8);
  c.force = NAN;
  EXPECT(bad(c, o64));
  c = chan(8, 8);
  c.visc_split = 0.5;
  c.tau0 = INFINITY;
  EXPECT(bad(c, o64));
  EXPECT(bad(chan(8, 8), osf));  // stress force with nn_pressure = 1
  lb_options obad = o64;
  obad.obs_every = 3;
  EXPECT(bad(chan(8, 8), obad));
  EXPECT(lb_workspace_bytes(nullptr, 1, &o64, &b) == LB_EINVAL);
  EXPECT(lb_workspace_bytes(cs.data(), 0, &o64, &b) == LB_EINVAL);
  EXPECT(lb_workspace_bytes(cs.data(), 1, nullptr, &b) == LB_EINVAL);
  EXPECT(lb_workspace_bytes(cs.data(), 1, &o64, nullptr) == LB_EINVAL);
  // lb_create failures before any device call
  lb_handle *h = nullptr;
  EXPECT(lb_create(cs.data(), 1, &o64, nullptr, 0, nullptr, &h) == LB_EINVAL && h == nullptr);
  EXPECT(lb_create(cs.data(), 1, &o64, reinterpret_cast<void *>(4096 + 8), 1 << 30, nullptr, &h) == LB_EINVAL);
  EXPECT(lb_create(cs.data(), 1, &o64, reinterpret_cast<void *>(4096), 16, nullptr, &h) == LB_ENOMEM);
  EXPECT(lb_create(cs.data(), 1, &o64, reinterpret_cast<void *>(4096), 1 << 30, nullptr, nullptr) == LB_EINVAL);
  EXPECT(lb_destroy(nullptr) == LB_OK);
  EXPECT(std::strcmp(lb_last_error(nullptr), "NULL handle") == 0);
  EXPECT(std::strcmp(lb_status_string(LB_EUNSTABLE), "LB_EUNSTABLE") == 0);
  EXPECT(std::strcmp(lb_status_string(12345), "unknown status") == 0);
  EXPECT(lb_step(nullptr, 1) == LB_EINVAL);
  double out = 0;
  EXPECT(lb_observe(nullptr, 0, 0, &out, 1) == LB_EINVAL);
  std::printf("host checks: %d failed\n", fails);
  return fails ? 1 : 0;
}
