// Stress driver for the HIP backend's host code on the stub runtime, built
// with -fsanitize=thread.  Every completion mechanism, several dispatcher
// threads, skewed submission (steals and retargeted jobs), DMA input copies
// issued at bind on input-copy streams, captured templates defined while
// another template's jobs run, the comparison modes, and batched vector
// jobs.  Every job's output header is checked (magic, canaries, job id, tag,
// a worker and slot of the context).  Exit status 0 = every check held;
// ThreadSanitizer reports races itself, and the stub counts graph-executable
// updates that overlapped a queued or running launch of the same executable.
#include <atomic>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"
#include "set.h"

namespace {

struct Run {
  const char* name;
  int mode, workers, slots, callback, dispatchers, policy, copy, copy_streams, inflight;
  int define_while_running;  // define captured templates while the jobs run
  int stress;                // 1: poison-fill slots after each job and delay each job's first stage
  int cb_streams;            // event chaining: callback streams (0 = one shared by every worker)
};

int run_images(const Run& r, int producers, int per_producer) {
  set_config cfg;
  std::memset(&cfg, 0, sizeof(cfg));
  cfg.abi_version = SET_ABI_VERSION;
  cfg.mode = r.mode;
  cfg.backend = SET_BACKEND_HIP;
  cfg.num_workers = r.workers;
  cfg.slots_per_worker = r.slots;
  cfg.work_stealing = 1;
  cfg.callback_mode = r.callback;
  cfg.submit_policy = r.policy;
  cfg.dispatch_threads = r.dispatchers;
  cfg.input_copy_streams = r.copy_streams;
  cfg.inflight_per_worker = r.inflight;
  cfg.callback_streams = r.cb_streams;
  cfg.staging_capacity = 256;
  cfg.batch_size = r.mode == SET_MODE_BATCH_SYNC ? r.workers : 0;
  set_ctx* c = nullptr;
  if (set_ctx_create(&cfg, &c) != SET_OK) {
    std::printf("%s: create failed: %s\n", r.name, set_last_error(nullptr));
    return 1;
  }
  set_job_template t;
  std::memset(&t, 0, sizeof(t));
  t.pipeline = SET_PIPE_BOX_HIST_U8;
  t.width = 32;
  t.height = 24;
  t.copy_mode = (uint32_t)r.copy;
  if (r.stress) {
    t.flags |= SET_TF_POISON;
    t.stress_delay_us = 20;
  }
  int tid = -1;
  if (set_template_define(c, &t, &tid) != SET_OK) {
    std::printf("%s: define failed: %s\n", r.name, set_last_error(c));
    return 2;
  }
  uint64_t in_b = 0, out_b = 0;
  set_job_io_bytes(c, tid, 0, &in_b, &out_b);
  const int total = producers * per_producer;
  const size_t stride = (out_b + 63) / 64 * 64;
  std::vector<char> in(in_b * 8 + 64), out(stride * total + 64);
  for (size_t i = 0; i < in.size(); ++i) in[i] = (char)(i * 7);
  std::vector<std::thread> th;
  std::atomic<int> submit_err{0};
  // ids are consecutive in submission order only within one producer, so
  // each producer owns a contiguous range of outputs and tags
  std::vector<uint64_t> ids(total);
  for (int p = 0; p < producers; ++p) {
    th.emplace_back([&, p] {
      for (int i = 0; i < per_producer; ++i) {
        const int k = p * per_producer + i;
        set_job_args a;
        std::memset(&a, 0, sizeof(a));
        a.host_in = in.data() + (size_t)(k % 8) * in_b;
        a.in_bytes = in_b;
        a.host_out = out.data() + (size_t)k * stride;
        a.out_bytes = out_b;
        a.worker_hint = -1;
        a.user_tag = (uint64_t)k;
        uint64_t id = 0;
        if (set_submit(c, tid, &a, 0, &id) != SET_OK) submit_err.fetch_add(1);
        ids[k] = id;
      }
    });
  }
  std::thread definer([&] {
    for (int k = 0; k < r.define_while_running; ++k) {
      set_job_template t2 = t;
      t2.flags = SET_TF_CAPTURE;
      t2.width = 16 + 8 * k;
      int id = -1;
      if (set_template_define(c, &t2, &id) != SET_OK) {
        std::printf("%s: define while running failed: %s\n", r.name, set_last_error(c));
        submit_err.fetch_add(1);
      }
    }
  });
  for (auto& x : th) x.join();
  definer.join();
  int rc = 0;
  if (set_drain(c, -1) != SET_OK) {
    std::printf("%s: drain failed: %s\n", r.name, set_last_error(c));
    rc = 3;
  }
  set_stats st;
  set_get_stats(c, &st);
  int bad = 0;
  for (int k = 0; k < total; ++k) {
    const set_out_header* h = reinterpret_cast<const set_out_header*>(out.data() + (size_t)k * stride);
    if (h->magic != SET_OUT_MAGIC || h->canary_ok != 1 || h->job_id != ids[k] || h->user_tag != (uint64_t)k ||
        (int)h->worker >= r.workers || (int)h->slot >= r.slots)
      ++bad;
  }
  if (bad || st.completed != (uint64_t)total || st.failed || submit_err.load()) {
    std::printf("%s: completed %llu of %d, failed %llu, %d wrong outputs, %d submit errors\n", r.name,
                (unsigned long long)st.completed, total, (unsigned long long)st.failed, bad, submit_err.load());
    rc = 4;
  }
  if (r.mode == SET_MODE_SET && r.policy == SET_SUBMIT_SKEW0 && r.workers > 1 && st.stolen == 0) {
    std::printf("%s: no steals under skewed submission\n", r.name);
    rc = 5;
  }
  std::printf("%-34s jobs %d stolen %llu\n", r.name, total, (unsigned long long)st.stolen);
  set_ctx_destroy(c);
  return rc;
}

int run_vectors() {
  set_config cfg;
  std::memset(&cfg, 0, sizeof(cfg));
  cfg.abi_version = SET_ABI_VERSION;
  cfg.mode = SET_MODE_SET;
  cfg.backend = SET_BACKEND_HIP;
  cfg.num_workers = 4;
  cfg.slots_per_worker = 4;
  cfg.work_stealing = 1;
  cfg.callback_mode = SET_CB_HOST_FLAG;
  cfg.dispatch_threads = 2;
  set_ctx* c = nullptr;
  if (set_ctx_create(&cfg, &c) != SET_OK) return 1;
  static float pool[1 << 16];
  set_job_template t;
  std::memset(&t, 0, sizeof(t));
  t.pipeline = SET_PIPE_SAXPY_BATCH_F32;
  t.max_n = 1 << 14;
  t.dev_x_pool = pool;
  t.dev_y_pool = pool;
  t.pool_len = 1 << 16;
  t.batch_max = 16;
  t.tiles_max = 256;
  int tid = -1;
  if (set_template_define(c, &t, &tid) != SET_OK) {
    std::printf("vectors: define failed: %s\n", set_last_error(c));
    return 2;
  }
  std::vector<set_vec_job> jobs(300);
  for (size_t i = 0; i < jobs.size(); ++i) jobs[i] = set_vec_job{64 * i, 32 * i, 1 + (i * 37) % 16000, 1.0f, 0};
  std::vector<float> res(jobs.size());
  uint64_t nb = 0;
  int rc = 0;
  for (int rep = 0; rep < 3 && rc == 0; ++rep)
    if (set_run_vector_jobs(c, tid, jobs.data(), jobs.size(), res.data(), nullptr, &nb) != SET_OK) {
      std::printf("vectors: %s\n", set_last_error(c));
      rc = 3;
    }
  std::printf("%-34s jobs %zu batches %llu\n", "set, vector batches", jobs.size(), (unsigned long long)nb);
  set_ctx_destroy(c);
  return rc;
}

}  // namespace

int main() {
  const Run runs[] = {
      {"set, event poll, 1 dispatcher", SET_MODE_SET, 4, 4, SET_CB_EVENT_POLL, 1, SET_SUBMIT_ROUND_ROBIN,
       SET_COPY_KERNELS, 0, 0, 0},
      {"set, event poll, 4 dispatchers, skew", SET_MODE_SET, 8, 4, SET_CB_EVENT_POLL, 4, SET_SUBMIT_SKEW0,
       SET_COPY_KERNELS, 0, 0, 0},
      {"set, host flag, 4 dispatchers, skew", SET_MODE_SET, 8, 4, SET_CB_HOST_FLAG, 4, SET_SUBMIT_SKEW0,
       SET_COPY_KERNELS, 0, 0, 0},
      {"set, event chain, 3 dispatchers", SET_MODE_SET, 6, 4, SET_CB_EVENT_CHAIN, 3, SET_SUBMIT_SKEW0,
       SET_COPY_NODES, 0, 0, 0},
      {"set, event chain, 2 callback streams", SET_MODE_SET, 6, 4, SET_CB_EVENT_CHAIN, 3, SET_SUBMIT_SKEW0,
       SET_COPY_KERNELS, 0, 0, 0, 0, 2},
      {"set, event chain, stream per worker", SET_MODE_SET, 6, 4, SET_CB_EVENT_CHAIN, 2, SET_SUBMIT_ROUND_ROBIN,
       SET_COPY_KERNELS, 0, 0, 0, 0, 6},
      {"set, same stream, 2 dispatchers", SET_MODE_SET, 4, 4, SET_CB_SAME_STREAM, 2, SET_SUBMIT_ROUND_ROBIN,
       SET_COPY_KERNELS, 0, 0, 0},
      {"set, event blocking, 4 dispatchers", SET_MODE_SET, 8, 4, SET_CB_EVENT_BLOCKING, 4, SET_SUBMIT_SKEW0,
       SET_COPY_KERNELS, 0, 0, 0},
      {"set, DMA at bind, 2 copy streams", SET_MODE_SET, 8, 4, SET_CB_EVENT_POLL, 4, SET_SUBMIT_SKEW0,
       SET_COPY_ASYNC_IN, 2, 1, 0},
      {"set, DMA on worker streams", SET_MODE_SET, 8, 16, SET_CB_EVENT_POLL, 1, SET_SUBMIT_ROUND_ROBIN,
       SET_COPY_ASYNC_IN, 0, 1, 0},
      {"set, host flag, define while running", SET_MODE_SET, 4, 4, SET_CB_HOST_FLAG, 2, SET_SUBMIT_ROUND_ROBIN,
       SET_COPY_KERNELS, 0, 0, 3},
      {"set, event chain, define while running", SET_MODE_SET, 4, 4, SET_CB_EVENT_CHAIN, 2, SET_SUBMIT_SKEW0,
       SET_COPY_KERNELS, 0, 0, 3},
      {"set, poison + delay, DMA at bind", SET_MODE_SET, 8, 2, SET_CB_EVENT_POLL, 4, SET_SUBMIT_SKEW0,
       SET_COPY_ASYNC_IN, 2, 1, 0, 1},
      {"set, poison + delay, host flag", SET_MODE_SET, 4, 1, SET_CB_HOST_FLAG, 2, SET_SUBMIT_SKEW0,
       SET_COPY_KERNELS, 0, 0, 0, 1},
      {"sync", SET_MODE_SYNC, 4, 1, 0, 1, 0, SET_COPY_ASYNC_IN, 2, 0, 0},
      {"graph", SET_MODE_GRAPH, 4, 1, 0, 1, 0, SET_COPY_KERNELS, 0, 0, 0},
      {"batch-sync", SET_MODE_BATCH_SYNC, 4, 2, 0, 1, 0, SET_COPY_NODES, 0, 0, 0},
      {"batch-sync, poison + delay", SET_MODE_BATCH_SYNC, 4, 2, 0, 1, 0, SET_COPY_KERNELS, 0, 0, 0, 1},
      {"queue model", SET_MODE_QUEUE, 4, 1, 0, 1, 0, SET_COPY_KERNELS, 0, 0, 0},
  };
  int rc = 0, i = 0;
  for (const Run& r : runs) {
    if (run_images(r, 3, r.mode == SET_MODE_SET ? 1500 : 200) != 0) rc |= 1 << i;
    ++i;
  }
  if (run_vectors() != 0) rc |= 1 << i;
  const uint64_t hz = hipstub::updates_while_in_flight();
  std::printf("stub: %llu launches, %llu executable updates overlapping a launch of the same executable\n",
              (unsigned long long)hipstub::launches(), (unsigned long long)hz);
  if (hz) rc |= 1 << 30;
  std::printf("tsan hip stress rc=%d\n", rc);
  return rc;
}
