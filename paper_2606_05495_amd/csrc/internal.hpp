// Internal declarations shared by the scheduler core, the HIP backend and the
// CPU fake backend.  Nothing here is part of the C ABI.
#pragma once

#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "set.h"
#include "tiles.hpp"

namespace setrt {

inline uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Message that set_last_error(NULL) returns on the calling thread (calls
// that have no context: a failed set_ctx_create, the no-allocation call).
void set_thread_error(const std::string& msg);

// Threads per block of the vector-batch work-item kernel of template t.
inline int vec_batch_block(const set_job_template& t) { return t.block > 0 ? t.block : kBlock; }

constexpr int kMaxWorkers = 256;     // b: workers (streams) of a context
constexpr int kMaxThreads = 64;      // dispatcher threads, input-copy streams
constexpr int kStatWorkers = 64;     // workers whose launches set_stats lists
constexpr int kMaxSlots = 64;
constexpr int kMaxTemplates = 16;
constexpr int kMaxStages = 40;
constexpr int kMaxHotspotSteps = 32;  // thermal-grid template: steps per job (one kernel each)

// Per-job scalar arguments.  Passed by value to the first kernel of a chain
// (a kernel-node placeholder, Section 4.1) and written by it into the slot's
// device header, where later stages read it.
struct JobScalars {
  uint64_t job_id;
  uint64_t seq;
  uint64_t user_tag;
  uint64_t n;
  uint64_t x_off;
  uint64_t y_off;
  uint32_t worker;
  uint32_t slot;
  float a;
  uint32_t flags;
};
static_assert(sizeof(JobScalars) == 64, "JobScalars layout");

// Device-side slot header (first bytes of every slot).  The first stage of a
// job writes job_id/seq/worker/slot/user_tag; the last stage copies them into
// the output header after checking the head and tail canaries.
struct DevSlotHdr {
  uint64_t canary_head;
  uint64_t job_id;
  uint64_t seq;
  uint64_t user_tag;
  uint32_t worker;
  uint32_t slot;
  uint64_t n;  // job length (vector / scan pipelines), read by later stages
  uint32_t pad[4];
};
static_assert(sizeof(DevSlotHdr) == 64, "DevSlotHdr layout");
static_assert(sizeof(set_out_header) == 64, "set_out_header layout");
static_assert(sizeof(set_config) == 104, "set_config layout");
static_assert(sizeof(set_job_template) == 96, "set_job_template layout");

// Descriptor table of a vector batch (host-written, copied to the slot by
// the batch's H2D): a 64-byte header, then one 48-byte descriptor per job.
// Each job carries its own work-item size, so one batch may mix size buckets
// while every job's result still depends only on (n, its item size).
struct VecBatchHdr {
  uint32_t count;        // jobs in the batch
  uint32_t total_tiles;  // work items in the batch
  uint32_t pad[14];
};
struct VecBatchDesc {
  uint64_t x_off, y_off;
  uint32_t n;
  float a;
  uint32_t tile_start;   // first work item of this job (non-decreasing)
  uint32_t ntiles;       // ceil(n / tile_elems)
  uint32_t tile_elems;   // elements per work item, multiple of 1024
  uint32_t pad[3];
};
static_assert(sizeof(VecBatchHdr) == 64, "VecBatchHdr layout");
static_assert(sizeof(VecBatchDesc) == 48, "VecBatchDesc layout");

inline uint64_t canary_value(int tmpl, int w, int s, int which) {
  return 0x5E7CA9A200000000ull ^ ((uint64_t)which << 60) ^ ((uint64_t)tmpl << 24) ^ ((uint64_t)w << 12) ^
         (uint64_t)s;
}

// A submitted job (M5 of the method: id, prepared parameters, is_stolen).
struct JobRec {
  uint64_t id;
  int tmpl;
  set_job_args args;
  int worker;     // worker whose slot the job is bound to
  int slot;       // bound slot
  int stolen;     // retargeted by a thief (Algorithm 2)
  uint64_t seq;   // binding sequence number of that slot
  uint64_t footprint;
  uint64_t t_submit, t_launch, t_done;
  int status;
  int64_t serve_ref;  // serving: request index (>= 0), vector batch -(2 + ring entry), or -1
  JobRec* next;   // free list / intrusive links
};

// Sizes one template needs, computed on the host.
struct TemplateSizes {
  uint64_t slot_bytes;
  int num_stages;
  uint64_t stage_bytes[kMaxStages];
  char stage_names[kMaxStages][32];
};

// Static per-job sizes of a template (in/out bytes for a job with length n).
uint64_t pipeline_in_bytes(const set_job_template& t, uint64_t n);
uint64_t pipeline_out_bytes(const set_job_template& t, uint64_t n);
int pipeline_validate(const set_job_template& t, std::string* why);
int pipeline_validate_job(const set_job_template& t, const set_job_args& a, std::string* why);
// Implemented by the HIP pipeline code (needs kernel tile constants); the fake
// backend uses the same sizes so footprints agree.
int pipeline_sizes(const set_job_template& t, TemplateSizes* out);
SlotLayout slot_layout(const set_job_template& t);

// Completion hook the scheduler core hands to a backend launch.
using DoneFn = void (*)(void* ctx, JobRec* job, int status);

// Execution backend: owns device resources of every template.
class Backend {
 public:
  virtual ~Backend() {}
  // Create per-worker resources (streams are borrowed or created here).
  virtual int init(const set_config& cfg, std::string* err) = 0;
  // Allocate/lay out slots and build per-slot graphs (SET/GRAPH) or the batch graph (BATCH_SYNC).
  virtual int define_template(int id, const set_job_template& t, std::string* err) = 0;
  // UpdateGraphParams(J, i): bind job to slot (worker, slot) of its template.
  virtual int bind(JobRec* job, std::string* err) = 0;
  // GraphLaunch + AddCallback: launch the bound slot's executable on the
  // worker's stream and arrange for done(ctx, job, status) after it finishes.
  virtual int launch(JobRec* job, DoneFn done, void* ctx, std::string* err) = 0;
  // Queue model: launch the bound slot's executable and record its completion
  // event without any callback; is_done() queries that event.
  virtual int launch_polled(JobRec* job, std::string* err) = 0;
  virtual int is_done(JobRec* job, bool* done, std::string* err) = 0;
  // Baselines, run on the caller's thread.
  virtual int run_sync(JobRec* job, int stream_index, std::string* err) = 0;
  virtual int run_graph(JobRec* job, int stream_index, std::string* err) = 0;
  virtual int run_batch(JobRec** jobs, int count, std::string* err) = 0;
  virtual int time_stage(int tmpl, int stage, int worker, int reps, double* avg_us, std::string* err) = 0;
  // A plain device copy of `bytes` (half read, half written), cold; see set_time_device_copy.
  virtual int time_device_copy(uint64_t bytes, int reps, double* avg_us, std::string* err) = 0;
  virtual uint64_t host_ns_sync() const { return 0; }
  // Pinned host staging owned by the library (descriptor tables, results).
  virtual void* alloc_host(uint64_t bytes) = 0;
  virtual void free_host(void* p) = 0;
  virtual void shutdown() = 0;
};

Backend* make_hip_backend();
Backend* make_fake_backend();

}  // namespace setrt
