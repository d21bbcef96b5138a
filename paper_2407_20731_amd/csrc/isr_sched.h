// Host-side runtime pieces: arena, sizes, pipeline entry points, scheduler.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "isr.h"
#include "isr_arena.h"
#include "isr_internal.h"

namespace isr {

// Sizes and scratch layout of one compression.
struct Sizes {
  u64 nv = 0;        // values per component
  int W = 0;         // bitmap words per element
  long long tiles = 0;
  int vbytes = 8;
  size_t off_histE = 0, off_histN = 0, off_histR = 0, off_histL = 0, off_st = 0, off_ticket = 0,
         off_lookback = 0, off_lists = 0, off_histEs = 0, off_histNs = 0, off_done = 0, off_lidx = 0, off_cnt = 0,
         off_slotsA = 0, off_slotsB = 0, off_chunk = 0;
  bool fast = false;         // streaming path
  int tile = 0;              // its dense-tile shape (elements per wavefront tile); 0 = wave-tile engine
  int gA = 0, gB = 0, xh = 0;  // its grids (workgroups per component) and extraction headroom
  long long sample_stride = 0;
  size_t zero_bytes = 0;     // leading scratch bytes to clear
  u64 list_cap = 0;
  size_t scratch_bytes = 0;
  size_t blob_max = 0;       // worst-case blob allocation
};
// full_lists: candidate lists for every value (no overflow possible); else a
// first-attempt capacity of an eighth of the values (at least 2^20), which the
// sampled window rarely exceeds; an overflow sets ST_LIST and the request is
// rerun with full lists.
Sizes plan_sizes(const isr_field* f, int tile, bool full_lists = true);
int ctx_tile(const isr_ctx* c, int order, int precision);

int enqueue_pipeline(isr_ctx* c, const Job& j, const Sizes& z, hipStream_t s, hipEvent_t* ev, bool fast);
int run_compress(isr_ctx* c, const isr_field* f, isr_blob** out, isr_stats* st, double cut_scale = 1.0);
int run_compress_quantized(isr_ctx* c, const isr_field* f, double share, isr_blob** out, isr_stats* st);
int run_batch(isr_ctx* c, const isr_field* fs, int count, isr_blob** outs, isr_stats* st);
int run_batch_sequential(isr_ctx* c, const isr_field* fs, int count, isr_blob** outs, isr_stats* st);
uint64_t request_footprint(const isr_field* f);
// isr_compress_noalloc: one compression with caller-provided scratch (at most
// scratch_cap bytes, used from its start) and the serialized blob written to
// d_out; no allocation of any kind.
int run_compress_noalloc(isr_ctx* c, const isr_field* f, char* scratch, size_t scratch_cap, void* d_out,
                         uint64_t out_cap, uint64_t* out_bytes, isr_stats* st);
// set the calling thread's isr_last_error() text and return code
int set_error(int code, const char* fmt, ...);
// Hybrid lossless stage (isr_lossless.cpp): a context's packer codes blobs on
// host threads, after copying each to pinned memory on the packer's stream.
struct Packer;
Packer* packer_create(int device, int threads);
void packer_destroy(Packer* p);
int packer_submit(Packer* p, const unsigned char* hdr, size_t hb, const void* dev_body, size_t body, int codec,
                  int level, uint32_t flags, uint64_t* job);
int packer_poll(Packer* p, uint64_t job, int wait_ms, void* out, uint64_t cap, uint64_t* out_bytes, double* secs);
int ctx_device(const isr_ctx* c);
Arena* ctx_arena(isr_ctx* c);
int ctx_max_inflight(const isr_ctx* c);
uint64_t ctx_budget(const isr_ctx* c);

// One compression in flight: its allocations, job, stream and completion event.
struct Task {
  isr_ctx* c = nullptr;
  double cut_scale = 1.0;  // the cut's share of the budget (quantised variant)
  isr_field f;
  Sizes z;
  char* scratch = nullptr;
  isr_blob* b = nullptr;
  Job j;
  hipStream_t s = nullptr;
  CompState* hs = nullptr;   // pinned copy of the per-component state
  hipEvent_t done = nullptr; // recorded after the state copy
  hipEvent_t ev[8] = {};
  bool timing = false;
  bool fast = false;         // this attempt runs the streaming path
  bool full_lists = false;   // candidate lists sized for every value (after an overflow)
  int iters = 0;
  float repair_ms = 0.f;
  double t_start = 0;
  isr_stats st;
};
int task_begin(isr_ctx* c, const isr_field* f, hipStream_t s, bool timing, Task* t);
int task_step(Task* t, isr_blob** out);
void task_release(Task* t);

// Continuous batching behind isr_submit / isr_poll.  A scheduler thread admits
// queued requests while a slot (max_inflight streams) and HBM budget are free,
// each admitted request runs its whole pipeline on its own stream so the
// kernels of different requests overlap on the device, and completions are
// retired (and their memory reused) as soon as their event fires.
class Scheduler {
 public:
  explicit Scheduler(isr_ctx* c);
  ~Scheduler();
  int submit(const isr_field* f, uint64_t* req);
  int poll(uint64_t req, int wait_ms, isr_blob** out, isr_stats* st);
  uint64_t admitted_high_water() const { return high_; }

 private:
  struct Req {
    uint64_t id = 0;
    isr_field f;
    double t_submit = 0;
    hipEvent_t ready = nullptr;  // producer stream's state at submit time (after the copy, if any)
    void* copy = nullptr;        // copy-on-submit: the library's copy of the field (and Jacobians)
    bool done = false;
    int status = 0;
    isr_blob* blob = nullptr;
    isr_stats st;
  };
  struct Slot {
    hipStream_t s = nullptr;
    bool busy = false;
    uint64_t id = 0;
    Task t;
  };
  void loop();
  bool admit_locked();
  void release_copy(Req& r);
  isr_ctx* ctx_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<uint64_t> queue_;
  std::map<uint64_t, Req> reqs_;
  std::vector<Slot> slots_;
  uint64_t next_id_ = 1;
  uint64_t high_ = 0;
  bool stop_ = false;
  std::thread worker_;
};

}  // namespace isr
