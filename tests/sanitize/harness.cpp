// Host-side checks of libjpet under AddressSanitizer and UndefinedBehaviorSanitizer: argument
// validation, plan enumeration, workspace layouts and batch layouts over many geometries, through
// the C-ABI only.  Built with the device launchers stubbed out (stubs.cpp); no GPU is touched.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "jpet.h"

static int failures = 0;
#define EXPECT(c)                                                    \
  do {                                                               \
    if (!(c)) {                                                      \
      printf("FAILED line %d: %s\n", __LINE__, #c);                 \
      ++failures;                                                    \
    }                                                                \
  } while (0)

static uint64_t lcg = 0x9e3779b97f4a7c15ull;
static double uniform(double a, double b) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return a + (b - a) * (double)(lcg >> 11) / 9007199254740992.0;
}

static jpet_geometry geometry(double R, double L, double sz, double sdl, double pix, int ny, int nz) {
  jpet_geometry g;
  memset(&g, 0, sizeof(g));
  g.R = R;
  g.L = L;
  g.sigma_z = sz;
  g.sigma_dl = sdl;
  g.pixel = pix;
  g.n_y = ny;
  g.n_z = nz;
  return g;
}

static void check_plans(jpet_geometry g, int64_t n) {
  size_t bytes = 0;
  if (jpet_mlem_workspace_size(&g, n, &bytes) != JPET_OK) return;  // out of domain: nothing more to check
  jpet_launch_info info;
  EXPECT(jpet_mlem_launch_info(&g, n, &info) == JPET_OK);
  int32_t count = 0;
  EXPECT(jpet_mlem_plan_candidates(&g, 0, nullptr, n, nullptr, nullptr, 0, &count) == JPET_OK);
  std::vector<int32_t> codes(count > 0 ? count : 1);
  std::vector<double> cost(codes.size());
  EXPECT(jpet_mlem_plan_candidates(&g, 0, nullptr, n, codes.data(), cost.data(), count, &count) == JPET_OK);
  EXPECT(count >= 1 && codes[0] == info.plan);
  for (int32_t k = 0; k < count; ++k) {
    jpet_geometry gk = g;
    gk.plan = codes[k];
    jpet_launch_info ik;
    EXPECT(jpet_mlem_launch_info(&gk, n, &ik) == JPET_OK && ik.plan == codes[k]);
    size_t b = 0;
    EXPECT(jpet_mlem_workspace_size(&gk, n, &b) == JPET_OK && b > 0);
    if (k > 0) EXPECT(cost[k] >= cost[k - 1]);
  }
  size_t tb = 0;
  EXPECT(jpet_mlem_tune_workspace_size(&g, n, codes.data(), count, &tb) == JPET_OK && tb >= bytes);
  // log-likelihood plans
  int32_t lcount = 0;
  EXPECT(jpet_mlem_plan_candidates(&g, 1, nullptr, n, nullptr, nullptr, 0, &lcount) == JPET_OK);
  size_t lb = 0;
  // the log-likelihood is defined for one sigma_z shared by all events
  EXPECT(jpet_loglik_workspace_size(&g, nullptr, n, &lb) == (g.sigma_z_edge == 0.0 ? JPET_OK : JPET_ENOTSUP));
  // every malformed code is refused the same way
  const int32_t bad[] = {-1, 4, 7, 1 | (5 << 3), 1 | (1 << 3) | (6 << 6), 1 | (1 << 3) | (3 << 12), 1 | (1 << 14)};
  for (int32_t c : bad) {
    jpet_geometry gb = g;
    gb.plan = c;
    EXPECT(jpet_mlem_workspace_size(&gb, n, &bytes) == JPET_EINVAL);
  }
}

int main() {
  // named workloads: 64^2 / 400^2 / 200^2 / 1024^2 / the paper's setting, and event counts 0..2^31-1
  const jpet_geometry named[] = {geometry(450, 500, 10, 63, 4, 64, 64), geometry(450, 500, 10, 63, 2, 400, 400),
                                 geometry(450, 500, 10, 63, 2.5, 200, 200), geometry(450, 1000, 5, 30, 0.5, 1024, 1024),
                                 geometry(130, 300, 10, 40, 4, 64, 76)};
  const int64_t counts[] = {0, 1, 7, 20000, 600000, 10000000, 2147483647};
  for (const jpet_geometry& g : named)
    for (int64_t n : counts) check_plans(g, n);
  // random geometries, including ones only the generic pass fits and ones out of domain
  for (int t = 0; t < 300; ++t) {
    jpet_geometry g = geometry(uniform(50, 600), uniform(100, 1200), uniform(0.5, 40), uniform(3, 120),
                               uniform(0.05, 8), (int)uniform(1, 2048), (int)uniform(1, 2048));
    g.kernel_variant = (int)uniform(0, 2);
    g.sigma_z_edge = uniform(0, 1) < 0.3 ? uniform(0, 1) : 0.0;
    check_plans(g, (int64_t)uniform(0, 2e7));
  }
  // batches: a layout for each mix of grids and resolutions, with fake device pointers (never used)
  for (int t = 0; t < 20; ++t) {
    const int count = 1 + (int)uniform(0, 64);
    std::vector<jpet_instance> inst(count);
    for (int k = 0; k < count; ++k) {
      const int n = (int[]){128, 256, 512}[(int)uniform(0, 3)];
      inst[k].g = geometry(450, 500, uniform(8, 15), uniform(40, 90), 600.0 / n, n, n);
      inst[k].events = (const float*)0x1000;
      inst[k].n = (int64_t)exp(uniform(log(5e4), log(2e6)));
      inst[k].s = nullptr;
      inst[k].rho = (float*)0x2000;
    }
    size_t bytes = 0;
    EXPECT(jpet_mlem_batched_workspace_size(inst.data(), count, &bytes) == JPET_OK && bytes > 0);
  }
  // argument validation
  jpet_geometry g = named[1];
  size_t b = 0;
  EXPECT(jpet_mlem_workspace_size(nullptr, 10, &b) == JPET_EINVAL);
  EXPECT(jpet_mlem_workspace_size(&g, -1, &b) == JPET_EINVAL);
  EXPECT(jpet_mlem_batched_workspace_size(nullptr, 3, &b) == JPET_EINVAL);
  EXPECT(jpet_mlem_batched_graph_create(nullptr, 0, 0, nullptr, 0, 0, nullptr, nullptr) == JPET_EINVAL);
  EXPECT(jpet_mlem_batched_graph_destroy(nullptr) == JPET_OK);
  printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
