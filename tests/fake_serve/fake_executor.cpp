// A fake executor for the serving core (test infrastructure, built by
// tests/test_serve_core.py with g++; no device code).  Hierarchies are
// bookkeeping entries of the size the request names; the "device work" is
// delegated to two callbacks: `check` inspects a request's data when it is
// prepared and names the number of V-cycles it will need (0: it converges in
// its cascade), `solve` writes its result when it leaves.  Every executor call
// is logged so that tests can follow admission, batching and completion.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "serve_core.h"

extern "C" {
typedef int (*fake_check_fn)(const inpaint_problem* p, int* cycles);
typedef int (*fake_solve_fn)(const inpaint_problem* p, double tol);
}

namespace {

using namespace inpaint;

struct FakeJob : ExecJob {
  int need = 0, cycles = 0;
};

struct Counter {
  std::mutex mu;
  size_t live = 0, peak = 0;
};

struct FakeHier : ExecHier {
  size_t n = 0;
  Counter* c = nullptr;
  ~FakeHier() override {
    std::lock_guard<std::mutex> g(c->mu);
    c->live -= n;
  }
};

class FakeExecutor : public Executor {
 public:
  FakeExecutor(fake_check_fn check, fake_solve_fn solve, int max_cycles)
      : check_(check), solve_(solve), max_cycles_(max_cycles) {}

  void start() override {
    std::unique_lock<std::mutex> lk(hold_mu_);
    hold_cv_.wait(lk, [&] { return !held_; });
  }

  void release_hold() {
    std::lock_guard<std::mutex> g(hold_mu_);
    held_ = false;
    hold_cv_.notify_all();
  }

  void describe(const inpaint_problem& p, std::string* shape, size_t* hier_bytes,
                size_t* stage_bytes) override {
    if (!p.f || !p.mask || !p.out) fail(INPAINT_E_INVALID, "NULL pointer argument");
    if (p.W < 1 || p.H < 1 || p.channels < 1 || p.channels > 4) fail(INPAINT_E_INVALID, "bad shape");
    *shape = std::to_string(p.W) + "x" + std::to_string(p.H) + "x" + std::to_string(p.channels);
    *hier_bytes = 4096 + (size_t)p.W * p.H * p.channels * 16;
    *stage_bytes = 0;
  }

  std::unique_ptr<ExecHier> create(const ServeRequest& r) override {
    auto h = std::make_unique<FakeHier>();
    h->n = r.hier_bytes;
    h->c = &bytes_;
    {
      std::lock_guard<std::mutex> g(bytes_.mu);
      bytes_.live += h->n;
      bytes_.peak = std::max(bytes_.peak, bytes_.live);
    }
    note("create " + r.shape + " for " + std::to_string(r.ticket));
    return h;
  }

  size_t bytes(const ExecHier& h) override { return static_cast<const FakeHier&>(h).n; }
  bool needs_staging(const ExecHier&, const ServeRequest&) override { return false; }

  void prepare(const std::vector<ServeRequest*>& fresh, const std::vector<ExecHier*>&) override {
    for (ServeRequest* r : fresh) {
      auto job = std::make_unique<FakeJob>();
      const int st = check_(&r->p, &job->need);
      r->job = std::move(job);
      if (st < 0) {
        r->status = st;
        r->msg = "rejected by the fake executor's check";
      }
      note("prepare " + std::to_string(r->ticket) + " " + std::to_string(st));
    }
  }

  void step(const std::vector<ServeRequest*>& cas, const std::vector<ServeRequest*>& going) override {
    std::string s = "step cas";
    for (ServeRequest* r : cas) s += " " + std::to_string(r->ticket);
    s += " going";
    for (ServeRequest* r : going) s += " " + std::to_string(r->ticket);
    note(s);
    for (ServeRequest* r : cas) r->leaving = job(r).need == 0;
    for (ServeRequest* r : going) {
      FakeJob& j = job(r);
      ++j.cycles;
      r->leaving = j.cycles >= j.need || j.cycles >= max_cycles_;
    }
  }

  void finish(const std::vector<ServeRequest*>& out) override {
    for (ServeRequest* r : out) {
      FakeJob& j = job(r);
      std::memset(&r->stats, 0, sizeof r->stats);
      r->stats.cycles = j.cycles;
      if (j.cycles < j.need) {
        r->status = INPAINT_NOT_CONVERGED;
        r->msg = "cycle cap reached before the tolerance";
      } else {
        const int st = solve_(&r->p, r->tol);
        r->status = st;
        if (st < 0) r->msg = "the fake executor failed this request";
      }
      note("finish " + std::to_string(r->ticket) + " " + std::to_string(r->status));
    }
  }

  std::string log() {
    std::lock_guard<std::mutex> g(log_mu_);
    return log_;
  }
  size_t peak() {
    std::lock_guard<std::mutex> g(bytes_.mu);
    return bytes_.peak;
  }

 private:
  static FakeJob& job(ServeRequest* r) { return *static_cast<FakeJob*>(r->job.get()); }
  void note(const std::string& s) {
    std::lock_guard<std::mutex> g(log_mu_);
    log_ += s + "\n";
  }

  fake_check_fn check_;
  fake_solve_fn solve_;
  int max_cycles_;
  std::mutex hold_mu_;
  std::condition_variable hold_cv_;
  bool held_ = true;
  std::mutex log_mu_;
  std::string log_;
  Counter bytes_;
};

struct FakeServer {
  FakeExecutor* ex = nullptr;  // owned by core
  std::unique_ptr<ServeCore> core;
};

}  // namespace

extern "C" {

// The loop waits in Executor::start until fake_server_release.
int fake_server_create(int max_batch, size_t budget, int max_cycles, fake_check_fn check,
                       fake_solve_fn solve, void** out) {
  return guarded([&] {
    auto ex = std::make_unique<FakeExecutor>(check, solve, max_cycles);
    auto* s = new FakeServer();
    s->ex = ex.get();
    s->core = std::make_unique<ServeCore>(std::move(ex), max_batch, budget);
    *out = s;
    return INPAINT_OK;
  });
}

void fake_server_release(void* s) { static_cast<FakeServer*>(s)->ex->release_hold(); }

int fake_server_submit(void* s, const inpaint_problem* p, double tol, uint64_t* ticket) {
  return guarded([&] {
    *ticket = static_cast<FakeServer*>(s)->core->submit(*p, tol);
    return INPAINT_OK;
  });
}

int fake_server_collect(void* s, uint64_t ticket, inpaint_stats* st, int block) {
  return guarded([&] { return static_cast<FakeServer*>(s)->core->collect(ticket, st, block != 0); });
}

const char* fake_server_last_error(void) { return g_err.c_str(); }

size_t fake_server_log(void* s, char* buf, size_t n) {
  const std::string l = static_cast<FakeServer*>(s)->ex->log();
  if (buf && n) {
    const size_t k = std::min(n - 1, l.size());
    std::memcpy(buf, l.data(), k);
    buf[k] = 0;
  }
  return l.size();
}

size_t fake_server_peak_bytes(void* s) { return static_cast<FakeServer*>(s)->ex->peak(); }

void fake_server_destroy(void* s) {
  auto* fs = static_cast<FakeServer*>(s);
  fs->ex->release_hold();
  delete fs;
}

}  // extern "C"
