// Stress driver for the scheduler core on the CPU fake backend, built with
// -fsanitize=thread: several producer threads, skewed submission (forcing
// steals), out-of-order completion callbacks, several configurations.
// Exit status 0 = every invariant held (ThreadSanitizer reports races itself).
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "set.h"

static int run(int mode, int b, int d, int policy, int stealing, int reorder, int producers, int per_producer,
               int dispatchers = 1, int extra_templates = 0, int steal_policy = SET_STEAL_ANY) {
  set_config cfg;
  std::memset(&cfg, 0, sizeof(cfg));
  cfg.abi_version = SET_ABI_VERSION;
  cfg.mode = mode;
  cfg.backend = SET_BACKEND_FAKE;
  cfg.num_workers = b;
  cfg.slots_per_worker = d;
  cfg.work_stealing = stealing;
  cfg.submit_policy = policy;
  cfg.fake_reorder_callbacks = reorder;
  cfg.staging_capacity = 64;
  cfg.dispatch_threads = dispatchers;
  cfg.steal_policy = steal_policy;
  set_ctx* c = nullptr;
  if (set_ctx_create(&cfg, &c) != SET_OK) {
    std::printf("create failed: %s\n", set_last_error(nullptr));
    return 1;
  }
  set_job_template t;
  std::memset(&t, 0, sizeof(t));
  t.pipeline = SET_PIPE_SAXPY_TANH_SUM_F32;
  t.max_n = 1 << 20;
  static float dummy[16];
  t.dev_x_pool = dummy;
  t.dev_y_pool = dummy;
  t.pool_len = 1ull << 24;
  int tid = -1;
  if (set_template_define(c, &t, &tid) != SET_OK) return 2;
  const int total = producers * per_producer;
  std::vector<set_out_header> outs(total);
  std::vector<std::thread> th;
  for (int p = 0; p < producers; ++p) {
    th.emplace_back([&, p] {
      for (int i = 0; i < per_producer; ++i) {
        const int k = p * per_producer + i;
        set_job_args a;
        std::memset(&a, 0, sizeof(a));
        a.host_out = &outs[k];
        a.out_bytes = sizeof(set_out_header) + 4;
        a.n = 1 + (k % 7) * 13;  // microseconds of simulated work
        a.a = 1.0f;
        a.worker_hint = -1;
        a.user_tag = (uint64_t)k;
        set_submit(c, tid, &a, 0, nullptr);
      }
    });
  }
  // templates defined while the producers' jobs are in flight
  std::thread definer([&] {
    for (int k = 0; k < extra_templates; ++k) {
      int id = -1;
      set_template_define(c, &t, &id);
    }
  });
  for (auto& x : th) x.join();
  definer.join();
  if (set_drain(c, -1) != SET_OK) return 3;
  set_stats st;
  set_get_stats(c, &st);
  int bad = 0;
  for (int k = 0; k < total; ++k)
    if (outs[k].magic != SET_OUT_MAGIC || outs[k].canary_ok != 1 || outs[k].user_tag != (uint64_t)k) ++bad;
  if (st.completed != (uint64_t)total || bad) {
    std::printf("mode %d: completed %llu of %d, %d bad outputs\n", mode, (unsigned long long)st.completed, total, bad);
    return 4;
  }
  if (mode == SET_MODE_SET && policy == SET_SUBMIT_SKEW0 && b > 1 && stealing && st.stolen == 0) return 5;
  if (!stealing && st.stolen != 0) return 6;
  set_ctx_destroy(c);
  return 0;
}

int main() {
  int rc = 0;
  rc |= run(SET_MODE_SET, 4, 8, SET_SUBMIT_ROUND_ROBIN, 1, 1, 3, 400);
  rc |= run(SET_MODE_SET, 4, 8, SET_SUBMIT_SKEW0, 1, 1, 2, 400) << 1;
  rc |= run(SET_MODE_SET, 3, 4, SET_SUBMIT_SKEW0, 0, 0, 2, 200) << 2;
  rc |= run(SET_MODE_SET, 8, 16, SET_SUBMIT_SHORTEST, 1, 1, 4, 300) << 3;
  rc |= run(SET_MODE_SYNC, 4, 2, 0, 1, 0, 2, 100) << 4;
  rc |= run(SET_MODE_BATCH_SYNC, 4, 2, 0, 1, 0, 2, 100) << 5;
  rc |= run(SET_MODE_QUEUE, 4, 2, 0, 1, 0, 3, 200) << 6;
  rc |= run(SET_MODE_SET, 6, 8, SET_SUBMIT_SKEW0, 1, 1, 3, 300, 3) << 7;
  rc |= run(SET_MODE_SET, 4, 4, SET_SUBMIT_ROUND_ROBIN, 0, 1, 2, 200, 2) << 8;
  rc |= run(SET_MODE_SET, 4, 4, SET_SUBMIT_SKEW0, 1, 1, 2, 300, 2, 5) << 9;
  rc |= run(SET_MODE_SET, 8, 4, SET_SUBMIT_SKEW0, 1, 1, 3, 300, 8, 0, SET_STEAL_BUSY) << 10;
  rc |= run(SET_MODE_SET, 8, 4, SET_SUBMIT_ROUND_ROBIN, 1, 1, 3, 300, 8, 0, SET_STEAL_BUSY) << 11;
  std::printf("tsan stress rc=%d\n", rc);
  return rc;
}
