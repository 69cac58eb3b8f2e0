// Host-side engine of batched integration: a list of jobs, the set of jobs
// that advance together, its device job table and work-unit queue, and the
// captured iteration graphs.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "mcv.h"
#include "mcv_internal.h"

namespace mcv {

mcv_status check_tuning(const mcv_tuning& t);
mcv_tuning default_tuning();

struct Job {
  JobDev j;
  void* block = nullptr;  // the job's device block
  int64_t n_points = 0;   // calls per pass
  int iters = 0;          // completed passes
  bool live = false;
};

struct Engine {
  int device = 0, n_cu = 1, prec = 0;
  hipStream_t stream = nullptr;      // caller's stream: every launch and copy
  hipStream_t cap_stream = nullptr;  // private stream used only for graph capture
  mcv_tuning tune = default_tuning();
  std::vector<Job> jobs;
  // the current set: member job indices, their records with the set's
  // partial buffers, and the device-side view
  std::vector<int> set_members;
  std::vector<JobDev> set_jobs;
  JobSet js;
  void* table = nullptr;  // unit prefix, queue counter, job table, sample arguments
  size_t table_cap = 0;
  void* scratch = nullptr;  // per-unit partial buffers of every member
  size_t scratch_cap = 0;
  struct Graph {
    hipGraphExec_t exec = nullptr;
  };
  Graph graphs[4];  // by refine flags
  // events of each iteration: start, after allocation, after the sample
  // pass, end (graph replays record only start and end)
  struct Ev {
    hipEvent_t a = nullptr, c = nullptr, b = nullptr, d = nullptr;
    bool graphed = false;
  };
  std::vector<Ev> ev;

  ~Engine();
  mcv_status add_job(const mcv_problem* p, int64_t n_points, int* index);
  void remove_job(int index);
  mcv_status build_set(const std::vector<int>& listed);
  mcv_status enqueue_iteration(uint32_t what, hipStream_t s, hipEvent_t after_alloc,
                               hipEvent_t after_sample);
  mcv_status iterate(uint32_t what, bool use_graph);
  mcv_status timing(int iteration, double* iter_ms, double* sample_ms);
  mcv_status history(int index, double* out, int cap, int* n_iter);
  void free_set_buffers();
  void drop_graphs();
};

}  // namespace mcv
