// The serving loop without the device: tickets, the arrival-order queue,
// admission by free slot and HBM footprint, continuous batching, completion
// and the latency stamps.  An Executor does the device work; the core decides
// what runs when.  Host-only C++ (no HIP), so the same loop runs against the
// GPU executor of the library and against a fake executor in CPU tests.
//
// One loop iteration ("step"):
//   1. admission: requests are taken in arrival order while a slot (of
//      max_batch) is free and the request's hierarchy fits the budget: an
//      idle hierarchy of the same shape is reused, idle hierarchies of other
//      shapes are freed to make room; the first request that does not fit
//      stops admission (no overtaking);
//   2. the admitted requests are prepared (staging, coarse problems, input
//      checks); a request whose data is rejected completes with its error;
//   3. one step of the device work for everybody: the cascade of the newly
//      admitted requests and one V-cycle of the running ones, together;
//   4. requests that converged or reached the cycle cap leave: their results
//      are written and they complete (slot and hierarchy become free).
// A failure the executor throws (a device error) ends the loop: every request
// not yet complete fails with that status, and later submits are refused.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "errors.h"
#include "inpaint.h"

namespace inpaint {

// What an executor keeps for one request (its iteration state).
struct ExecJob {
  virtual ~ExecJob() = default;
};

// One device hierarchy of the server's pool; the executor frees its device
// memory in the destructor.
struct ExecHier {
  virtual ~ExecHier() = default;
  std::string shape;
};

struct ServeRequest {
  uint64_t ticket = 0;
  inpaint_problem p{};
  double tol = 0.0;
  std::string shape;                     // requests of one shape share hierarchies
  size_t hier_bytes = 0, stage_bytes = 0;  // stage_bytes: 0 for device-resident buffers
  double t_submit = 0.0, t_start = 0.0;
  bool done = false;
  int status = INPAINT_PENDING;
  std::string msg;     // with a failing status
  inpaint_stats stats{};
  int slot = -1;       // flag slot, in [0, max_batch)
  int pool_idx = -1;   // hierarchy in the pool
  bool leaving = false;  // set by Executor::step: converged or at the cycle cap
  std::unique_ptr<ExecJob> job;
};

class Executor {
 public:
  virtual ~Executor() = default;
  // First call on the loop thread.
  virtual void start() {}
  // On the submitting thread: validate the problem (throws Fail for a bad
  // argument), name its shape, the device bytes of its hierarchy and those of
  // the staging buffers it needs (0 when its buffers are device memory).
  virtual void describe(const inpaint_problem& p, std::string* shape, size_t* hier_bytes,
                        size_t* stage_bytes) = 0;
  // A new hierarchy for r's shape.
  virtual std::unique_ptr<ExecHier> create(const ServeRequest& r) = 0;
  // Device bytes hierarchy h holds now (with staging once it has some).
  virtual size_t bytes(const ExecHier& h) = 0;
  // Whether r would add its staging bytes to h (h has no staging yet).
  virtual bool needs_staging(const ExecHier& h, const ServeRequest& r) = 0;
  // Stage the newly admitted requests (hiers[i] is fresh[i]'s hierarchy); a
  // request whose data is rejected gets its status (< 0), msg and stats, the
  // others stay INPAINT_PENDING.
  virtual void prepare(const std::vector<ServeRequest*>& fresh,
                       const std::vector<ExecHier*>& hiers) = 0;
  // One step of device work: the cascade of cas and one V-cycle of going.
  // Sets `leaving` on the requests that converged or reached the cycle cap.
  virtual void step(const std::vector<ServeRequest*>& cas, const std::vector<ServeRequest*>& going) = 0;
  // Results of the requests that leave: write out, set status, msg and stats.
  virtual void finish(const std::vector<ServeRequest*>& out) = 0;
  // A request ended: drop what the executor kept for it.
  virtual void release(ServeRequest& r) { r.job.reset(); }
};

class ServeCore {
 public:
  ServeCore(std::unique_ptr<Executor> ex, int max_batch, size_t budget);
  // Finishes every submitted request, then stops the loop and frees the pool.
  ~ServeCore();
  ServeCore(const ServeCore&) = delete;
  ServeCore& operator=(const ServeCore&) = delete;

  // Queue a request; throws Fail (E_INVALID, E_NOMEM for a hierarchy larger
  // than the whole budget, or the status that broke the loop).
  uint64_t submit(const inpaint_problem& p, double tol);
  // The request's status once complete (stats copied, ticket forgotten);
  // INPAINT_PENDING while it runs and block is false.
  int collect(uint64_t ticket, inpaint_stats* st, bool block);
  size_t budget() const { return budget_; }

 private:
  double now_ms() const;
  int take_hier(ServeRequest& r);
  bool evict(size_t need, int keep);
  void complete(ServeRequest& r);
  void run();
  void loop();

  std::unique_ptr<Executor> ex_;
  const int max_batch_;
  const size_t budget_;
  std::chrono::steady_clock::time_point t0_;

  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  bool stop_ = false;
  int broken_ = 0;  // an inpaint_status once the loop failed
  std::string broken_msg_;
  uint64_t next_ticket_ = 1;
  std::deque<std::shared_ptr<ServeRequest>> queue_;
  std::map<uint64_t, std::shared_ptr<ServeRequest>> reqs_;

  // owned by the loop thread
  std::vector<std::unique_ptr<ExecHier>> pool_;
  std::vector<char> pool_busy_;
  size_t pool_bytes_ = 0;
  std::vector<int> free_slots_;

  std::thread th_;  // last: started once everything above is initialised
};

}  // namespace inpaint
