// Serving: the GPU executor of the serving core (serve_core.h) and the C ABI
// of the server.  The core queues requests, admits them by slot and HBM
// footprint and runs the continuous-batching loop; this executor does the
// device work of each step with the batched plans (batch.h): admitted requests
// are staged together, their cascades run in the same step as one V-cycle of
// the requests already running, and requests leave as soon as they converge.
// Each request runs the same arithmetic as a solve of it alone, so its result
// does not depend on the mix.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <map>

#include "batch.h"
#include "serve_core.h"

namespace inpaint {
namespace {

size_t staging_bytes(const inpaint_problem& p) {
  const size_t n = (size_t)p.W * p.H;
  return 2 * round_up(n * p.channels * sizeof(float), 256) + round_up(n, 256);
}

struct GpuJob : ExecJob {
  std::unique_ptr<Member> m;
};

struct GpuHier : ExecHier {
  std::unique_ptr<Workspace> ws;
};

Member& member(ServeRequest* r) { return *static_cast<GpuJob*>(r->job.get())->m; }

class GpuExecutor : public Executor {
 public:
  GpuExecutor(const Opts& o, int max_batch, int dev) : o_(o), max_batch_(max_batch), dev_(dev) {
    HIPCHK(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    HIPCHK(hipMalloc(&flags_dev_, (size_t)max_batch_ * kFlagInts * sizeof(int)));
    HIPCHK(hipHostMalloc(&flags_host_, (size_t)max_batch_ * kFlagInts * sizeof(int),
                         hipHostMallocDefault));
  }

  ~GpuExecutor() override {
    int old = -1;
    (void)hipGetDevice(&old);
    (void)hipSetDevice(dev_);
    if (s_) (void)hipStreamSynchronize(s_);
    if (prep_dev_) (void)hipFree(prep_dev_);
    if (plan_dev_) (void)hipFree(plan_dev_);
    if (out_dev_) (void)hipFree(out_dev_);
    if (flags_dev_) (void)hipFree(flags_dev_);
    if (flags_host_) (void)hipHostFree(flags_host_);
    if (s_) (void)hipStreamDestroy(s_);
    if (old >= 0) (void)hipSetDevice(old);
  }

  void start() override { HIPCHK(hipSetDevice(dev_)); }

  void describe(const inpaint_problem& p, std::string* shape, size_t* hier_bytes,
                size_t* stage_bytes) override {
    validate_problem(p, -1, o_);
    const Key k = key(p);
    char s[96];
    std::snprintf(s, sizeof s, "%dx%dx%d", p.W, p.H, p.channels);
    *shape = s;
    {
      std::lock_guard<std::mutex> g(mu_);
      auto it = ws_size_.find(k);
      if (it == ws_size_.end()) it = ws_size_.emplace(k, workspace_bytes(k)).first;
      *hier_bytes = it->second;
    }
    *stage_bytes = (!is_device_ptr(p.f) || !is_device_ptr(p.mask) || !is_device_ptr(p.out))
                       ? staging_bytes(p)
                       : 0;
  }

  std::unique_ptr<ExecHier> create(const ServeRequest& r) override {
    auto h = std::make_unique<GpuHier>();
    h->ws = create_workspace(key(r.p));
    return h;
  }

  size_t bytes(const ExecHier& h) override {
    const Workspace& w = *static_cast<const GpuHier&>(h).ws;
    size_t b = w.bytes;
    if (w.stage_base) b += staging_bytes(inpaint_problem{nullptr, nullptr, w.key.W, w.key.H, w.key.C, nullptr});
    return b;
  }

  bool needs_staging(const ExecHier& h, const ServeRequest&) override {
    return !static_cast<const GpuHier&>(h).ws->stage_base;
  }

  void prepare(const std::vector<ServeRequest*>& fresh, const std::vector<ExecHier*>& hiers) override {
    std::vector<Member*> fm;
    for (size_t i = 0; i < fresh.size(); ++i) {
      ServeRequest* r = fresh[i];
      auto job = std::make_unique<GpuJob>();
      job->m.reset(new Member());
      Member& m = *job->m;
      m.idx = 0;
      m.slot = r->slot;
      r->job = std::move(job);
      init_member(m, r->p, static_cast<GpuHier*>(hiers[i])->ws.get(), o_, r->tol, s_);
      fm.push_back(&m);
    }
    Plan prep;
    build(prep, fm, [&] { build_prepare(prep, fm, o_, flags_dev_); });
    upload({&prep}, &prep_dev_, &prep_cap_, s_);
    HIPCHK(issue(prep, o_.prec, o_.B, s_));
    read_flags();
    for (ServeRequest* r : fresh) {
      Member& m = member(r);
      check_prepared(flags_host_, &m);
      if (m.status != INPAINT_OK) {
        r->status = m.status;
        r->msg = m.msg;
        fill_stats(&m, r->stats);
      }
    }
  }

  void step(const std::vector<ServeRequest*>& cas, const std::vector<ServeRequest*>& going) override {
    std::vector<Member*> cm, gm;
    for (ServeRequest* r : cas) cm.push_back(&member(r));
    for (ServeRequest* r : going) gm.push_back(&member(r));
    Plan pc, py;
    build(pc, cm, [&] {
      build_cascade(pc, cm, o_);
      add_gather(pc, cm, flags_dev_);
    });
    build(py, gm, [&] {
      build_cycle(py, gm, o_);
      add_gather(py, gm, flags_dev_);
    });
    for (Member* m : gm) ++m->cycles;
    account(cm, pc);
    account(gm, py);
    upload({&pc, &py}, &plan_dev_, &plan_cap_, s_);
    HIPCHK(issue(pc, o_.prec, o_.B, s_));
    HIPCHK(issue(py, o_.prec, o_.B, s_));
    read_flags();
    apply_flags(flags_host_, cm, pc);
    apply_flags(flags_host_, gm, py);
    auto mark = [&](const std::vector<ServeRequest*>& rs, const std::vector<Member*>& ms, const Plan& P) {
      for (size_t i = 0; i < rs.size(); ++i)
        if (ms[i]->done || ms[i]->cycles >= o_.max_cycles) {
          finish_member(ms[i], P.cur0[i]);
          rs[i]->leaving = true;
        }
    };
    mark(cas, cm, pc);
    mark(going, gm, py);
  }

  void finish(const std::vector<ServeRequest*>& out) override {
    std::vector<Member*> ms;
    for (ServeRequest* r : out) ms.push_back(&member(r));
    Plan po;
    build_output(po, ms);
    upload({&po}, &out_dev_, &out_cap_, s_);
    HIPCHK(issue(po, o_.prec, o_.B, s_));
    for (Member* m : ms)
      if (m->out_host)
        HIPCHK(hipMemcpyAsync(m->out, m->o_d, (size_t)m->W * m->H * m->C * sizeof(float),
                              hipMemcpyDeviceToHost, s_));
    HIPCHK(hipStreamSynchronize(s_));
    for (ServeRequest* r : out) {
      Member& m = member(r);
      r->status = m.status;
      r->msg = m.msg;
      fill_stats(&m, r->stats);
    }
  }

 private:
  Key key(const inpaint_problem& p) const {
    return Key{dev_, p.W, p.H, p.channels, o_.B, o_.o, coarsest_side(o_.B), o_.prec};
  }

  void read_flags() {
    HIPCHK(hipMemcpyAsync(flags_host_, flags_dev_, (size_t)max_batch_ * kFlagInts * sizeof(int),
                          hipMemcpyDeviceToHost, s_));
    HIPCHK(hipStreamSynchronize(s_));
  }

  const Opts o_;
  const int max_batch_;
  const int dev_;
  hipStream_t s_ = nullptr;
  int* flags_dev_ = nullptr;
  int* flags_host_ = nullptr;
  unsigned char* prep_dev_ = nullptr;
  size_t prep_cap_ = 0;
  unsigned char* plan_dev_ = nullptr;
  size_t plan_cap_ = 0;
  unsigned char* out_dev_ = nullptr;
  size_t out_cap_ = 0;
  std::mutex mu_;                  // describe() runs on the submitting threads
  std::map<Key, size_t> ws_size_;  // workspace bytes per key (host-side sizes only)
};

}  // namespace
}  // namespace inpaint

using namespace inpaint;

struct inpaint_server {
  std::unique_ptr<ServeCore> core;
};

extern "C" {

#define INPAINT_EXPORT __attribute__((visibility("default")))

INPAINT_EXPORT int inpaint_server_create(const inpaint_server_cfg* cfg, inpaint_server** srv) {
  return guarded([&] {
    if (!srv) fail(INPAINT_E_INVALID, "NULL server pointer");
    *srv = nullptr;
    if (cfg && cfg->struct_size != (int)sizeof(inpaint_server_cfg))
      fail(INPAINT_E_INVALID, "inpaint_server_cfg.struct_size must equal sizeof(inpaint_server_cfg)");
    Opts o = resolve(cfg && cfg->opts.struct_size ? &cfg->opts : nullptr);
    o.profile = 0;
    if (cg_schedule(o.schedule))
      fail(INPAINT_E_INVALID, "the server runs the multigrid schedules (CG is a comparison schedule)");
    if (o.schedule == INPAINT_SCHED_WARM)
      fail(INPAINT_E_INVALID, "the server solves from the cascade (its outputs hold no guess)");
    int max_batch = 64;
    if (cfg && cfg->max_batch) max_batch = cfg->max_batch;
    if (max_batch < 1 || max_batch > 1024) fail(INPAINT_E_INVALID, "max_batch must lie in [1, 1024]");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    const size_t budget = (cfg && cfg->hbm_budget) ? cfg->hbm_budget : fr / 10 * 8;
    auto ex = std::make_unique<GpuExecutor>(o, max_batch, dev);
    std::unique_ptr<inpaint_server> sv(new inpaint_server());
    sv->core = std::make_unique<ServeCore>(std::move(ex), max_batch, budget);
    *srv = sv.release();
    return INPAINT_OK;
  });
}

INPAINT_EXPORT int inpaint_server_submit(inpaint_server* srv, const inpaint_problem* p, double tol,
                                         uint64_t* ticket) {
  return guarded([&] {
    if (!srv || !p || !ticket) fail(INPAINT_E_INVALID, "NULL pointer argument");
    *ticket = srv->core->submit(*p, tol);
    return INPAINT_OK;
  });
}

INPAINT_EXPORT int inpaint_server_poll(inpaint_server* srv, uint64_t ticket, inpaint_stats* st) {
  return guarded([&] {
    if (!srv) fail(INPAINT_E_INVALID, "NULL server");
    return srv->core->collect(ticket, st, false);
  });
}

INPAINT_EXPORT int inpaint_server_wait(inpaint_server* srv, uint64_t ticket, inpaint_stats* st) {
  return guarded([&] {
    if (!srv) fail(INPAINT_E_INVALID, "NULL server");
    return srv->core->collect(ticket, st, true);
  });
}

INPAINT_EXPORT void inpaint_server_destroy(inpaint_server* srv) {
  if (!srv) return;
  delete srv;  // the core finishes the submitted requests, then frees the pool and the executor
}

}  // extern "C"
