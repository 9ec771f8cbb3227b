// Concurrency check of the serving loop under ThreadSanitizer: four submitting
// threads (some waiting on their tickets), one thread draining completions and
// reading statistics, against a simulated device.  A ticket is reported once, so a
// wait may find its ticket already drained (ZPM_ENOTFOUND); every other outcome must
// be success.  Exit status 0 when every request succeeded.
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "zpm.h"

int main() {
  zpm_server_config cfg{};
  cfg.hbm_budget = 1ull << 30;
  cfg.n_streams = 3;
  cfg.max_batch = 64;
  zpm_server *s = nullptr;
  if (zpm_server_create_simulated(&cfg, 1e11, 2e-5, -1, &s) != ZPM_OK) return 2;
  static uint64_t fake[4];   // never dereferenced by the simulated device
  std::atomic<int> bad{0};
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t) {
    th.emplace_back([&, t] {
      for (int i = 0; i < 300; ++i) {
        zpm_job j{};
        j.a = fake;
        j.b = fake;
        j.c = fake + 1;
        j.da = j.db = 16 + (t * 37 + i) % 500;
        j.Na = j.Nb = 64 + i % 300;
        j.wc = (zpm_out_bits(j.da, j.Na, j.db, j.Nb) + 63) / 64;
        uint64_t tk;
        if (zpm_server_submit(s, &j, &tk) != ZPM_OK) {
          ++bad;
          continue;
        }
        if (i % 3) continue;
        int32_t st;
        double lat;
        const int rc = zpm_server_wait(s, tk, 10.0, &st, &lat);
        if (rc == ZPM_ENOTFOUND) continue;
        if (rc != ZPM_OK || st != ZPM_OK) ++bad;
      }
    });
  }
  std::thread drain([&] {
    uint64_t tk[256];
    int32_t st[256];
    double lat[256];
    int64_t n;
    for (int k = 0; k < 2000; ++k) {
      if (zpm_server_completions(s, tk, st, lat, 256, &n) != ZPM_OK) ++bad;
      for (int64_t i = 0; i < n; ++i)
        if (st[i] != ZPM_OK) ++bad;
      zpm_server_report r;
      if (zpm_server_stats(s, &r) != ZPM_OK) ++bad;
    }
  });
  for (auto &x : th) x.join();
  drain.join();
  zpm_server_destroy(s);
  std::printf("failures %d\n", bad.load());
  return bad.load() ? 1 : 0;
}
