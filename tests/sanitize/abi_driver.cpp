// Host-side driver of the C ABI's argument validation, built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitizers.py).
// Every call here must be rejected before any device work, so it runs without a
// GPU; the sanitizers abort on any invalid memory access or undefined behaviour
// in the validation layer.
#include <cstdio>
#include <cstring>

#include "rl.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s (%s)\n", what, rl_last_error());
    ++failures;
  }
}

int main() {
  rl_plan out = reinterpret_cast<rl_plan>(0x1234);
  const int64_t bad_shapes[][3] = {{0, 8, 8},    {8, -1, 8},    {8, 8, 7},   {8, 8, 2},
                                   {8, 8, 22},   {8, 22, 8},    {8, 8, 70},  {8, 105, 8},
                                   {8, 8, 8192}, {8192, 8, 8},  {8, 8, 4096}};
  for (const auto& sh : bad_shapes) {
    rl_status st = rl_plan_create(sh, reinterpret_cast<const float*>(4096), 0, &out);
    expect(st == RL_E_INVALID || st == RL_E_UNSUPPORTED, "bad shape rejected");
    expect(out == nullptr, "*out cleared");
  }
  const int64_t sh[3] = {8, 8, 8};
  expect(rl_plan_create(nullptr, reinterpret_cast<const float*>(4096), 0, &out) == RL_E_INVALID,
         "NULL shape");
  expect(rl_plan_create(sh, nullptr, 0, &out) == RL_E_INVALID, "NULL psf");
  expect(rl_plan_create(sh, reinterpret_cast<const float*>(4100), 0, &out) == RL_E_INVALID,
         "misaligned psf");
  expect(rl_plan_create(sh, reinterpret_cast<const float*>(4096), 7, &out) == RL_E_INVALID,
         "unknown boundary");
  expect(rl_plan_create(sh, reinterpret_cast<const float*>(4096), 0, nullptr) == RL_E_INVALID,
         "NULL out");
  rl_options opt;
  std::memset(&opt, 0, sizeof(opt));
  opt.precision = 9;
  expect(rl_plan_create_ex(sh, reinterpret_cast<const float*>(4096), 0, &opt, &out) ==
             RL_E_INVALID, "unknown precision");
  std::memset(&opt, 0, sizeof(opt));
  opt.psf_shape[0] = 9;
  opt.psf_shape[1] = 8;
  opt.psf_shape[2] = 8;
  expect(rl_plan_create_ex(sh, reinterpret_cast<const float*>(4096), 0, &opt, &out) ==
             RL_E_INVALID, "psf larger than the volume");
  std::memset(&opt, 0, sizeof(opt));
  opt.x_elems = 5;
  expect(rl_plan_create_ex(sh, reinterpret_cast<const float*>(4096), 0, &opt, &out) ==
             RL_E_INVALID, "x_elems");
  const int64_t big[3] = {8, 8, 3000};
  expect(rl_plan_create(big, reinterpret_cast<const float*>(4096), RL_BOUNDARY_ZERO, &out) ==
             RL_E_UNSUPPORTED, "zero boundary grid too large");
  const float* psfs[2] = {reinterpret_cast<const float*>(4096), nullptr};
  const int64_t shapes[6] = {8, 8, 8, 8, 8, 8};
  expect(rl_plan_create_batch(2, shapes, psfs, 0, nullptr, &out) == RL_E_INVALID, "NULL psf in batch");
  expect(rl_plan_create_batch(0, shapes, psfs, 0, nullptr, &out) == RL_E_INVALID, "empty batch");

  // handles are checked against the live set, never dereferenced
  rl_plan fake = reinterpret_cast<rl_plan>(0x1234560);
  double d[4];
  int n = 0;
  char name[64];
  int64_t thr = 0;
  expect(rl_iterate(fake, nullptr, nullptr, 1) == RL_E_INVALID, "fake handle iterate");
  expect(rl_iterate_noalloc(fake, nullptr, nullptr, 1) == RL_E_INVALID, "fake handle noalloc");
  expect(conv3d_fft(fake, nullptr, nullptr) == RL_E_INVALID, "fake handle conv");
  expect(rl_plan_get_flux(fake, d, 4, &n) == RL_E_INVALID, "fake handle flux");
  expect(rl_plan_get_alpha(fake, d, 4, &n) == RL_E_INVALID, "fake handle alpha");
  expect(rl_plan_get_pass_kernel(fake, RL_KERNEL_Y, name, sizeof(name), &thr) == RL_E_INVALID,
         "fake handle pass kernel");
  rl_stop_rule rule;
  std::memset(&rule, 0, sizeof(rule));
  rule.metric = RL_STOP_FSC;
  expect(rl_iterate_stop(fake, nullptr, nullptr, 3, &rule) == RL_E_INVALID, "fake handle stop");
  expect(rl_fsc(fake, nullptr, nullptr, 8, 0.1, d, nullptr) == RL_E_INVALID, "fake handle fsc");
  expect(rl_ssim(fake, nullptr, nullptr, d) == RL_E_INVALID, "fake handle ssim");
  rl_plan_destroy(nullptr);
  rl_plan_destroy(fake);
  const int64_t odd[3] = {3, 4, 4};
  expect(rl_split_diagonal(reinterpret_cast<const float*>(4096), odd,
                           reinterpret_cast<float*>(4096), reinterpret_cast<float*>(4096),
                           nullptr) == RL_E_INVALID, "odd split");
  expect(rl_probe_copy(reinterpret_cast<void*>(4096), reinterpret_cast<void*>(8192), 10,
                       nullptr) == RL_E_INVALID, "copy size");
  for (int s = -1; s <= 7; ++s) expect(rl_status_string(static_cast<rl_status>(s)) != nullptr,
                                       "status string");
  // without a device, a valid request stops at the device check
  const int64_t good[3] = {8, 16, 32};
  rl_status st = rl_plan_create(good, reinterpret_cast<const float*>(4096), 0, &out);
  expect(st == RL_E_DEVICE || st == RL_E_INVALID, "valid shape reaches the device check");
  std::printf(failures ? "FAILED %d\n" : "OK\n", failures);
  return failures ? 1 : 0;
}
