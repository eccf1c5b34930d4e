// Host harness of libredsum's C ABI, run without a GPU, with the library's
// host code built under AddressSanitizer and UndefinedBehaviorSanitizer
// (hipcc -Xarch_host) by the test suite.  It drives the host-side paths
// that run before any HIP call or without one: argument validation of
// every entry point, the thread-local error messages, the plan tables, the
// tuner's candidate search with a cost callback, the probe formulas
// (Eq. 6-8), the no-device path (RED_ENODEV) and shutdown.  Exit status 0
// when every check holds (a sanitizer report aborts).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "redsum.h"

static int fails = 0;
#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #c, red_last_error()); \
      ++fails;                                                              \
    }                                                                       \
  } while (0)

static void* P(unsigned long v) { return reinterpret_cast<void*>(v); }

struct Seen {
  std::vector<red_plan> plans;
  int fail_at = -1;
};

static double fake_cost(red_plan* p, void* ctx) {
  Seen* s = static_cast<Seen*>(ctx);
  s->plans.push_back(*p);
  if ((int)s->plans.size() == s->fail_at) return (double)RED_EHIP;
  if (p->variant == RED_VARIANT_PERSISTENT && p->grid > 100) p->grid = 100;
  return 10.0 + p->grid / 100.0 + p->wg / 1000.0 + p->ipt / 10.0 + p->variant - (p->flags & 1) / 2.0;
}

int main() {
  double d = 0, e = 0, f = 0;
  int32_t n32 = 0;
  // validation before any HIP call
  CHECK(red_sum(99, nullptr, 0, nullptr, nullptr) == RED_EINVAL);
  CHECK(strlen(red_last_error()) > 0);
  CHECK(red_sum(RED_F32, nullptr, 10, P(64), nullptr) == RED_EINVAL);
  CHECK(red_sum(RED_F32, P(64), -1, P(64), nullptr) == RED_EINVAL);
  CHECK(red_sum(RED_F32, P(66), 4, P(64), nullptr) == RED_EINVAL);
  CHECK(red_sum(RED_F32, P(64), 4, P(68), nullptr) == RED_EINVAL);
  red_opts o;
  memset(&o, 0, sizeof o);
  o.plan = red_plan{RED_VARIANT_RELAUNCH, 100, 4, 0, 0};
  CHECK(red_sum_ex(RED_F32, P(64), 4, P(64), nullptr, &o) == RED_EINVAL);
  o.plan = red_plan{RED_VARIANT_RELAUNCH, 256, 3, 0, 0};
  CHECK(red_sum_ex(RED_F32, P(64), 4, P(64), nullptr, &o) == RED_EINVAL);
  o.plan = red_plan{RED_VARIANT_RELAUNCH, 256, 4, RED_NOALLOC_MAX_GRID + 1, 0};
  CHECK(red_sum_noalloc(RED_F32, P(64), 4, P(64), nullptr, &o) == RED_EINVAL);
  memset(&o, 0, sizeof o);
  o.flags = 1 << 20;
  CHECK(red_sum_ex(RED_F32, P(64), 4, P(64), nullptr, &o) == RED_EINVAL);
  CHECK(red_sum_segmented(nullptr, nullptr, 3, nullptr, nullptr) == RED_EINVAL);
  CHECK(red_sum_segmented(reinterpret_cast<const float*>(P(64)), reinterpret_cast<const int64_t*>(P(68)), 2,
                          reinterpret_cast<double*>(P(64)), nullptr) == RED_EINVAL);
  int64_t bad_off[3] = {0, 5, 2};
  CHECK(red_sum_segmented_loop(reinterpret_cast<const float*>(P(64)), bad_off, 2, reinterpret_cast<double*>(P(64)),
                               nullptr) == RED_EINVAL);
  CHECK(sync_bench_wave(9, 64, 10, &d, &e, nullptr, nullptr) == RED_EINVAL);
  CHECK(sync_bench_grid(0, 256, 10, &d, &e, nullptr, nullptr) == RED_EINVAL);
  CHECK(sync_bench_grid_r(8, 256, 0, 16, 16, 5, &d, &e, nullptr, nullptr) == RED_EINVAL);
  CHECK(sync_bench_grid_published(8, 256, -3, 0, 0, 5, &d, &e, nullptr, nullptr) == RED_EINVAL);
  int64_t nerr = 0;
  CHECK(sync_check_grid_visibility_published(0, 256, 0, 10, &nerr, nullptr) == RED_EINVAL);
  CHECK(sync_bench_relaunch_ex(8, 64, 0, 4, 4, 0, 10, &d, &e, nullptr, nullptr) == RED_EINVAL);
  CHECK(sync_bench_spin(0, 8, 1, 10, &d, &e, nullptr) == RED_EINVAL);
  double wbuf[64];
  CHECK(sync_check_wave(0, 9, wbuf, wbuf, nullptr) == RED_EINVAL);
  CHECK(sync_check_watchdog(4, 64, 9, 100, nullptr) == RED_EINVAL);
  CHECK(red_bw_proxy_ex(P(64), 1024, 4, 256, 2, nullptr) == RED_EINVAL);
  CHECK(stencil_jacobi_1d(reinterpret_cast<float*>(P(64)), reinterpret_cast<float*>(P(80)), 10, 1, 0.25f, 0,
                          nullptr, nullptr) == RED_EINVAL);
  CHECK(red_max_coresident(100, &n32) == RED_EINVAL);
  // a long message through the formatter
  char name[600];
  memset(name, 'x', sizeof name - 1);
  name[sizeof name - 1] = 0;
  CHECK(red_sum(RED_F32, P(64), (int64_t)1 << 41, P(64), nullptr) == RED_EINVAL);
  CHECK(strstr(red_last_error(), "out of range") != nullptr);

  // plan tables: round trip, and the default plan without a device
  red_plan p{RED_VARIANT_ATOMIC, 256, 2, 512, 1}, q;
  CHECK(red_set_plan(RED_BF16, RED_ACC_COMPENSATED, 1 << 20, &p) == RED_OK);
  CHECK(red_get_plan(RED_BF16, RED_ACC_COMPENSATED, (1 << 20) - 5, &q) == RED_OK);
  CHECK(q.variant == 2 && q.wg == 256 && q.ipt == 2 && q.grid == 512 && q.flags == 1);
  CHECK(red_get_plan(RED_F32, RED_ACC_COMPENSATED, 1000, &q) == RED_OK && q.variant == RED_VARIANT_SINGLE);
  CHECK(red_set_segmented_plan(1 << 17, &p) == RED_OK);
  CHECK(red_get_segmented_plan(1 << 17, &q) == RED_OK && q.grid == 512);
  red_plan bad{RED_VARIANT_SINGLE, 256, 4, 0, 0};
  CHECK(red_set_segmented_plan(5, &bad) == RED_EINVAL);

  // the tuner's search with a fake cost
  Seen seen;
  red_plan best;
  double best_us = 0;
  CHECK(red_autotune_search(RED_F32, (int64_t)1 << 28, 256, 8, 1, 0, fake_cost, &seen, &best, &best_us) == RED_OK);
  CHECK(seen.plans.size() == 264 && best_us > 0);
  Seen cut;
  cut.fail_at = 5;
  CHECK(red_autotune_search(RED_F32, (int64_t)1 << 28, 256, 8, 0, 0, fake_cost, &cut, &best, &best_us) == RED_EHIP);
  CHECK(cut.plans.size() == 5);
  Seen small;
  CHECK(red_autotune_search(RED_I32, 3000, 256, 8, 0, 9, fake_cost, &small, &best, &best_us) == RED_OK);
  CHECK(small.plans.size() == 9);
  CHECK(red_autotune_search(RED_I32, 3000, 0, 8, 0, 9, fake_cost, &small, &best, &best_us) == RED_EINVAL);

  // probe formulas
  CHECK(fabs(red_eq6_overhead(9000.0, 2000.0, 8, 1) - 1000.0) < 1e-9);
  CHECK(fabs(red_eq7_latency(5000.0, 1000.0, 4096, 512) - 4000.0 / 3584.0) < 1e-12);
  double a[6] = {10, 12, 11, 13, 9, 10.5}, b[6] = {5, 5.5, 4.5, 5, 6, 5.25};
  CHECK(red_eq8_sigma(a, b, 6, 64, 8) > 0);
  CHECK(isnan(red_eq8_sigma(a, b, 1, 64, 8)));

  // no device: the calls that pass validation report RED_ENODEV
  CHECK(red_init(0) == RED_ENODEV);
  CHECK(red_sum(RED_F32, P(64), 4, P(64), nullptr) == RED_ENODEV);
  CHECK(red_sum_noalloc(RED_F32, P(64), 4, P(64), nullptr, nullptr) == RED_ENODEV);
  CHECK(red_device_info(&n32, nullptr, nullptr, nullptr, nullptr, nullptr) == RED_ENODEV);
  red_shutdown();
  red_shutdown();
  (void)f;
  (void)name;
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("abi harness ok\n");
  return 0;
}
