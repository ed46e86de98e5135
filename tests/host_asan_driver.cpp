// Host-side driver of the C ABI for the AddressSanitizer test
// (tests/test_host_asan.py): the argument validation and the
// domain-contiguous row permutation of ecg_setup (also by Morton keys) run
// on the host before any device call, so an instrumented build exercises
// them without a GPU.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "ecg.h"

static int fails = 0;
static void expect(int got, int want, const char* what) {
  if (got != want) { std::printf("FAIL %s: %d (want %d) %s\n", what, got, want, ecg_last_error()); ++fails; }
}

int main() {
  ecg_opts o;
  ecg_opts_default(&o);
  const int nx = 30, ny = 20, n = nx * ny, px = 3, py = 2, t = px * py;
  std::vector<int32_t> rp(n + 1, 0), ci, dom(n);
  std::vector<double> v;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int r = i + nx * j;
      if (j > 0) { ci.push_back(r - nx); v.push_back(-1); }
      if (i > 0) { ci.push_back(r - 1); v.push_back(-1); }
      ci.push_back(r); v.push_back(4);
      if (i < nx - 1) { ci.push_back(r + 1); v.push_back(-1); }
      if (j < ny - 1) { ci.push_back(r + nx); v.push_back(-1); }
      rp[r + 1] = (int32_t)ci.size();
      dom[r] = (i * px) / nx + px * ((j * py) / ny);
    }
  ecg_ctx* c = nullptr;
  // invalid arguments
  expect(ecg_setup(nullptr, n, rp.data(), ci.data(), v.data(), dom.data(), t, 2, &o), ECG_EINVAL, "null out");
  expect(ecg_setup(&c, n, rp.data(), ci.data(), v.data(), dom.data(), 0, 2, &o), ECG_EINVAL, "t0");
  expect(ecg_setup(&c, n, rp.data(), ci.data(), v.data(), dom.data(), 65, 2, &o), ECG_EINVAL, "t65");
  expect(ecg_setup(&c, n, rp.data(), ci.data(), v.data(), dom.data(), t, 17, &o), ECG_EINVAL, "s17");
  {
    auto ci2 = ci; ci2[7] = n;
    expect(ecg_setup(&c, n, rp.data(), ci2.data(), v.data(), dom.data(), t, 2, &o), ECG_EINVAL, "col range");
    auto rp2 = rp; rp2[5] = rp2[7];
    expect(ecg_setup(&c, n, rp2.data(), ci.data(), v.data(), dom.data(), t, 2, &o), ECG_EINVAL, "rowptr");
    auto v2 = v; v2[3] = NAN;
    expect(ecg_setup(&c, n, rp.data(), ci.data(), v2.data(), dom.data(), t, 2, &o), ECG_EINVAL, "nan");
    auto d2 = dom; for (auto& d : d2) if (d == 4) d = 3;
    expect(ecg_setup(&c, n, rp.data(), ci.data(), v.data(), d2.data(), t, 2, &o), ECG_EINVAL, "empty domain");
    auto d3 = dom; d3[0] = t;
    expect(ecg_setup(&c, n, rp.data(), ci.data(), v.data(), d3.data(), t, 2, &o), ECG_EINVAL, "domain range");
    ecg_opts o2 = o; o2.ca = 3;
    expect(ecg_setup(&c, n, rp.data(), ci.data(), v.data(), dom.data(), t, 2, &o2), ECG_EINVAL, "ca");
    std::vector<int64_t> keys(n, 0);
    ecg_opts o4 = o; o4.permute_domains = 0; o4.row_key = keys.data();
    expect(ecg_setup(&c, n, rp.data(), ci.data(), v.data(), dom.data(), t, 2, &o4), ECG_EINVAL,
           "row_key without the domain order");
    expect(ecg_grid_morton_keys(nx, ny, 0, keys.data()), ECG_EINVAL, "morton nz0");
    expect(ecg_grid_morton_keys(nx, ny, 1, nullptr), ECG_EINVAL, "morton null");
  }
  // Morton keys of the grid (host code)
  std::vector<int64_t> mkeys(n, -1);
  expect(ecg_grid_morton_keys(nx, ny, 1, mkeys.data()), ECG_OK, "morton keys");
  // valid input in both row orders and with Morton keys: host validation
  // and the domain-contiguous permutation run; without a GPU the call then
  // reports ECG_EDEVICE
  for (int perm = 0; perm <= 2; ++perm) {
    ecg_opts o3 = o; o3.permute_domains = perm > 0;
    if (perm == 2) o3.row_key = mkeys.data();
    const int rc = ecg_setup(&c, n, rp.data(), ci.data(), v.data(), dom.data(), t, 2, &o3);
    if (rc == ECG_OK) ecg_destroy(c);
    else expect(rc, ECG_EDEVICE, "valid setup without a GPU");
  }
  expect(ecg_spmm_noalloc(nullptr, nullptr, nullptr, 4), ECG_EINVAL, "noalloc null");
  expect(ecg_set_preconditioner(nullptr, 1, nullptr), ECG_EINVAL, "precond null");
  for (int code = -4; code <= 3; ++code)
    if (!ecg_strerror(code)) { std::printf("FAIL strerror %d\n", code); ++fails; }
  ecg_destroy(nullptr);
  std::printf(fails ? "failures: %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
