// Host-only checks of the C ABI, built with AddressSanitizer and UndefinedBehaviorSanitizer
// around the library's host code (tests/test_sanitizers.py): every argument check that runs
// before device work, on a context created without a device.  Exit status 0 when every
// call returns the code the interface documents.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "twolink.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  if (got != want) {
    std::fprintf(stderr, "%s: got %d, want %d\n", what, got, want);
    failures++;
  }
}

int main() {
  tl_ctx* c = nullptr;
  expect(tl_create(&c, -1, nullptr), TL_OK, "host-only create");
  if (!c) return 2;
  void* fake = reinterpret_cast<void*>(0x10000);   // never dereferenced: validation stops first
  double* out = reinterpret_cast<double*>(0x30000);
  tl_geom g{{8, 6, 4, 4}}, bad{{8, 0, 4, 4}}, huge{{4096, 4096, 16, 1}};

  expect(tl_check_geom(&g), TL_OK, "geometry");
  expect(tl_check_geom(&bad), TL_ERR_SHAPE, "zero extent");
  expect(tl_check_geom(&huge), TL_ERR_SHAPE, "2^28 sites");
  expect(tl_check_geom(nullptr), TL_ERR_ARG, "NULL geometry");
  expect(tl_twolinks_bytes(&g, TL_F32, 4) == (size_t)4 * 3 * 192 * 72 ? 0 : 1, 0, "two-link bytes");
  expect(tl_twolinks_bytes(&g, 9, 1) == 0 ? 0 : 1, 0, "bad precision bytes");

  // build: shape, precision, slices
  int32_t rep[2] = {1, 1}, outside[2] = {1, 4}, ok[2] = {1, 3};
  expect(tl_build_twolinks(c, &bad, fake, nullptr, 0, TL_F32, fake), TL_ERR_SHAPE, "build bad geometry");
  expect(tl_build_twolinks(c, &g, fake, nullptr, 0, 9, fake), TL_ERR_PRECISION, "build bad precision");
  expect(tl_build_twolinks(c, &g, fake, rep, 2, TL_F32, fake), TL_ERR_ARG, "build repeated slice");
  expect(tl_build_twolinks(c, &g, fake, outside, 2, TL_F32, fake), TL_ERR_SHAPE, "build slice outside");
  expect(tl_build_twolinks(c, &g, fake, ok, 2, TL_F32, fake), TL_ERR_DEVICE, "build valid, no device");
  expect(tl_build_twolinks(c, &g, fake, nullptr, 0, TL_F32 | TL_ONELINK, fake), TL_ERR_PRECISION, "one-link to build");
  expect(tl_pack_links(c, &g, fake, nullptr, 0, TL_F32, fake), TL_ERR_PRECISION, "pack without one-link bit");
  expect(tl_pack_links(c, &g, fake, nullptr, 0, TL_BF16 | TL_W12 | TL_ONELINK, fake), TL_ERR_DEVICE, "pack valid");

  // laplacian: slice, overlap
  int32_t ws[1] = {2};
  char* a = reinterpret_cast<char*>(0x100000);
  expect(tl_laplacian(c, &g, fake, nullptr, 0, TL_F32, 4, a, a + (1 << 20)), TL_ERR_SHAPE, "laplacian t outside");
  expect(tl_laplacian(c, &g, fake, ws, 1, TL_F32, 1, a, a + (1 << 20)), TL_ERR_SHAPE, "laplacian t not in W");
  expect(tl_laplacian(c, &g, fake, nullptr, 0, TL_F32, 1, a, a + 64), TL_ERR_ARG, "laplacian overlap");
  expect(tl_laplacian(c, &g, fake, ws, 1, TL_F32, 2, a, a + (1 << 20)), TL_ERR_DEVICE, "laplacian valid");

  // plans and smearing: jobs, steps, sigma, flags; uneven batch with slice lists
  std::vector<int32_t> ts = {0, 1, 3}, ts2 = {0, 2}, wsl = {0, 1};
  tl_job jobs[2];
  std::memset(jobs, 0, sizeof jobs);
  jobs[0].g = g;
  jobs[0].W = fake;
  jobs[0].n_rhs = 3;
  jobs[0].t_of_rhs = ts.data();
  jobs[0].psi = fake;
  jobs[1] = jobs[0];
  jobs[1].n_rhs = 2;
  jobs[1].t_of_rhs = ts2.data();
  jobs[1].w_slices = wsl.data();
  jobs[1].n_w_slices = 2;
  tl_plan* p = nullptr;
  expect(tl_plan_create(c, jobs, 1, 10, 2.0, TL_F32, 0, &p), TL_ERR_DEVICE, "plan valid");
  expect(tl_plan_create(c, jobs, 0, 10, 2.0, TL_F32, 0, &p), TL_ERR_ARG, "plan no jobs");
  expect(tl_plan_create(c, jobs, 1, -1, 2.0, TL_F32, 0, &p), TL_ERR_ARG, "plan negative steps");
  expect(tl_plan_create(c, jobs, 1, 10, 7.0, TL_F32, 0, &p), TL_ERR_ARG, "plan sigma/n > 2/3");
  expect(tl_plan_create(c, jobs, 1, 12, 2.0, TL_F32 | TL_ONELINK, 0, &p), TL_ERR_DEVICE, "one-link plan valid");
  expect(tl_plan_create(c, jobs, 1, 10, 2.0, TL_F32 | TL_ONELINK, 0, &p), TL_ERR_ARG, "one-link sigma/n > 1/6");
  expect(tl_plan_create(c, jobs, 1, 10, 2.0, TL_F32, 16, &p), TL_ERR_ARG, "plan unknown flag");
  expect(tl_plan_create(c, jobs, 1, 10, 2.0, TL_F32, TL_ONE_STEP | TL_AUTOTUNE, &p), TL_ERR_DEVICE, "one-step flag valid");
  expect(tl_plan_create(c, jobs, 1, 10, 2.0, TL_F32, TL_PLAIN | TL_GRAPH, &p), TL_ERR_ARG, "plain with graph");
  expect(tl_plan_create(c, jobs, 2, 10, 2.0, TL_F32, 0, &p), TL_ERR_SHAPE, "RHS slice not in W");
  ts2[1] = 1;
  expect(tl_plan_create(c, jobs, 2, 10, 2.0, TL_F32, 0, &p), TL_ERR_DEVICE, "uneven batch valid");
  expect(tl_smear(c, jobs, 2, 10, 2.0, TL_BF16 | TL_W12, TL_GRAPH | TL_AUTOTUNE), TL_ERR_DEVICE, "smear valid");
  expect(p == nullptr ? 0 : 1, 0, "no plan returned");

  // reductions, the no-allocation form and the streaming probe
  expect(tl_reduce(c, 3, 10, 1, fake, nullptr, out), TL_ERR_ARG, "reduce bad kind");
  expect(tl_reduce(c, TL_DOT, 10, 1, fake, nullptr, out), TL_ERR_ARG, "dot needs phi");
  expect(tl_reduce(c, TL_NORM2, 10, 1, fake, nullptr, out), TL_ERR_DEVICE, "reduce valid");
  expect(tl_reduce_noalloc(c, TL_NORM2, 4096 * 64 + 1, 1024, fake, nullptr, out), TL_ERR_SHAPE, "no-alloc beyond area");
  expect(tl_reduce_noalloc(c, TL_NORM2, 4096 * 64, 1024, fake, nullptr, out), TL_ERR_DEVICE, "no-alloc full area");
  double ms = 0.0;
  expect(tl_stream_time(c, fake, 1 << 20, 4, 2, 0, 3, &ms), TL_ERR_DEVICE, "stream valid");
  expect(tl_stream_time(c, fake, 64, 4, 2, 0, 3, &ms), TL_ERR_ARG, "stream too small");

  tl_ctx_stats st;
  expect(tl_get_stats(c, &st), TL_OK, "stats");
  expect((int)(st.graphs_captured + st.tune_sweeps + st.tune_hits + st.smear_plan_hits), 0, "no device work counted");
  expect(tl_get_stats(c, nullptr), TL_ERR_ARG, "stats NULL");
  expect(tl_set_stream(c, nullptr), TL_OK, "set stream on a host-only context");
  expect(tl_sync(c), TL_ERR_DEVICE, "sync host-only");
  expect(std::strlen(tl_last_error(c)) > 0 ? 0 : 1, 0, "error message");
  expect(tl_destroy(c), TL_OK, "destroy");
  expect(tl_destroy(nullptr), TL_ERR_ARG, "destroy NULL");
  if (failures == 0) std::printf("abi host checks: all passed\n");
  return failures == 0 ? 0 : 1;
}
