// Serving: a request loop with continuous batching.  Requests are admitted in
// arrival order while a batch slot is free and their hierarchy fits the
// server's HBM budget; admitted requests join the running batch at the next
// V-cycle boundary (their staging and cascade run first) and leave it as soon
// as they converge, so requests that arrive while others run share every
// batched launch with them.  Each request runs the same arithmetic as a solve
// of it alone, so its result does not depend on the mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "batch.h"

namespace inpaint {
namespace {

struct Request {
  uint64_t ticket = 0;
  inpaint_problem p{};
  double tol = 0.0;
  Key key{};
  size_t ws_bytes = 0, stage_bytes = 0;  // stage_bytes: 0 for device-resident buffers
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
  bool done = false;
  int status = INPAINT_PENDING;
  inpaint_stats stats{};
  std::unique_ptr<Member> m;
  int pool_idx = -1;
};

size_t staging_bytes(const inpaint_problem& p) {
  const size_t n = (size_t)p.W * p.H;
  return 2 * round_up(n * p.channels * sizeof(float), 256) + round_up(n, 256);
}

}  // namespace
}  // namespace inpaint

using namespace inpaint;

struct inpaint_server {
  Opts o;
  int max_batch = 64;
  size_t budget = 0;
  int dev = 0;
  hipStream_t s = nullptr;
  std::chrono::steady_clock::time_point t0;
  std::thread th;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  int broken = 0;  // an inpaint_status once the loop failed
  std::string broken_msg;
  uint64_t next_ticket = 1;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> reqs;
  std::map<Key, size_t> ws_size;  // workspace bytes per key (host-side sizes only)

  // owned by the loop thread
  std::vector<std::unique_ptr<Workspace>> pool;
  std::vector<char> pool_busy;
  size_t pool_bytes = 0;
  int* flags_dev = nullptr;
  int* flags_host = nullptr;
  std::vector<int> free_slots;
  unsigned char* prep_dev = nullptr;
  size_t prep_cap = 0;
  unsigned char* plan_dev = nullptr;
  size_t plan_cap = 0;
  unsigned char* out_dev = nullptr;
  size_t out_cap = 0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }

  size_t pool_ws_bytes(const Workspace& w) const {
    size_t b = w.bytes;
    if (w.stage_base) b += staging_bytes(inpaint_problem{nullptr, nullptr, w.key.W, w.key.H, w.key.C, nullptr});
    return b;
  }

  // A free workspace for request r from the pool, evicting idle workspaces of
  // other shapes when the budget requires it; -1 if it cannot fit now.
  int take_ws(const Request& r) {
    for (size_t i = 0; i < pool.size(); ++i)
      if (!pool_busy[i] && pool[i] && pool[i]->key == r.key) {
        const size_t extra = (r.stage_bytes && !pool[i]->stage_base) ? r.stage_bytes : 0;
        if (pool_bytes + extra > budget && !evict(extra, (int)i)) return -1;
        pool_bytes += extra;
        pool_busy[i] = 1;
        return (int)i;
      }
    const size_t need = r.ws_bytes + r.stage_bytes;
    if (pool_bytes + need > budget && !evict(need, -1)) return -1;
    auto ws = create_workspace(r.key);
    pool_bytes += need;
    for (size_t i = 0; i < pool.size(); ++i)
      if (!pool[i]) {
        pool[i] = std::move(ws);
        pool_busy[i] = 1;
        return (int)i;
      }
    pool.push_back(std::move(ws));
    pool_busy.push_back(1);
    return (int)pool.size() - 1;
  }

  // Free idle workspaces (not `keep`) until `need` more bytes fit the budget.
  bool evict(size_t need, int keep) {
    for (size_t i = 0; i < pool.size() && pool_bytes + need > budget; ++i)
      if (pool[i] && !pool_busy[i] && (int)i != keep) {
        pool_bytes -= pool_ws_bytes(*pool[i]);
        pool[i].reset();
      }
    return pool_bytes + need <= budget;
  }

  void complete(Request& r, Member* m) {
    inpaint_stats st{};
    if (m) fill_stats(m, st);
    st.status = m ? m->status : r.status;
    st.t_submit_ms = r.t_submit;
    st.t_start_ms = r.t_start;
    st.t_done_ms = now_ms();
    if (m) {
      free_slots.push_back(m->slot);
      if (r.pool_idx >= 0) pool_busy[r.pool_idx] = 0;
    }
    std::lock_guard<std::mutex> g(mu);
    r.stats = st;
    r.status = st.status;
    r.done = true;
    cv_done.notify_all();
  }

  void run();
  void loop();
};

void inpaint_server::run() {
  try {
    loop();
  } catch (const Fail& e) {
    std::lock_guard<std::mutex> g(mu);
    broken = e.code;
    broken_msg = g_err;
  } catch (...) {
    std::lock_guard<std::mutex> g(mu);
    broken = INPAINT_E_DEVICE;
    broken_msg = "unexpected exception in the server loop";
  }
  // fail whatever is left
  std::lock_guard<std::mutex> g(mu);
  for (auto& kv : reqs)
    if (!kv.second->done) {
      kv.second->status = broken ? broken : INPAINT_E_DEVICE;
      kv.second->stats.status = kv.second->status;
      kv.second->done = true;
    }
  queue.clear();
  cv_done.notify_all();
}

void inpaint_server::loop() {
  HIPCHK(hipSetDevice(dev));
  std::vector<std::shared_ptr<Request>> active;  // prepared and cycling
  while (true) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
      if (stop && queue.empty() && active.empty()) return;
    }
    // admission: arrival order, while a slot is free and the hierarchy fits
    std::vector<std::shared_ptr<Request>> fresh;
    while (active.size() + fresh.size() < (size_t)max_batch) {
      std::shared_ptr<Request> r;
      {
        std::lock_guard<std::mutex> g(mu);
        if (queue.empty()) break;
        r = queue.front();
      }
      const int idx = take_ws(*r);
      if (idx < 0) break;
      {
        std::lock_guard<std::mutex> g(mu);
        queue.pop_front();
      }
      r->pool_idx = idx;
      fresh.push_back(r);
    }
    // staging, hierarchies and input checks of the admitted requests
    std::vector<Member*> cas;
    if (!fresh.empty()) {
      std::vector<Member*> fm;
      for (auto& r : fresh) {
        r->m.reset(new Member());
        Member& m = *r->m;
        m.idx = 0;
        m.slot = free_slots.back();
        free_slots.pop_back();
        init_member(m, r->p, pool[r->pool_idx].get(), o, r->tol, s);
        r->t_start = now_ms();
        fm.push_back(&m);
      }
      Plan prep;
      build(prep, fm, [&] { build_prepare(prep, fm, o, flags_dev); });
      upload({&prep}, &prep_dev, &prep_cap, s);
      HIPCHK(issue(prep, o.prec, o.B, s));
      HIPCHK(hipMemcpyAsync(flags_host, flags_dev, (size_t)max_batch * kFlagInts * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (auto& r : fresh) {
        check_prepared(flags_host, r->m.get());
        if (r->m->status != INPAINT_OK)
          complete(*r, r->m.get());
        else
          cas.push_back(r->m.get());
      }
    }
    // one step for everybody: the cascade of the new requests, one V-cycle of
    // the running ones
    std::vector<Member*> going;
    for (auto& r : active) going.push_back(r->m.get());
    Plan pc, py;
    build(pc, cas, [&] {
      build_cascade(pc, cas, o);
      add_gather(pc, cas, flags_dev);
    });
    build(py, going, [&] {
      build_cycle(py, going, o);
      add_gather(py, going, flags_dev);
    });
    for (Member* m : going) ++m->cycles;
    account(cas, pc);
    account(going, py);
    upload({&pc, &py}, &plan_dev, &plan_cap, s);
    HIPCHK(issue(pc, o.prec, o.B, s));
    HIPCHK(issue(py, o.prec, o.B, s));
    HIPCHK(hipMemcpyAsync(flags_host, flags_dev, (size_t)max_batch * kFlagInts * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    apply_flags(flags_host, cas, pc);
    apply_flags(flags_host, going, py);
    // requests that are finished leave the batch
    std::vector<std::shared_ptr<Request>> next, leaving;
    std::vector<Member*> out;
    auto sort_out = [&](std::vector<Member*>& ms, const Plan& P,
                        const std::vector<std::shared_ptr<Request>>& rs) {
      for (size_t i = 0; i < ms.size(); ++i) {
        Member* m = ms[i];
        std::shared_ptr<Request> r;
        for (auto& q : rs)
          if (q->m.get() == m) r = q;
        if (m->done || m->cycles >= o.max_cycles) {
          finish_member(m, P.cur0[i]);
          leaving.push_back(r);
          out.push_back(m);
        } else {
          next.push_back(r);
        }
      }
    };
    sort_out(cas, pc, fresh);
    sort_out(going, py, active);
    if (!out.empty()) {
      Plan po;
      build_output(po, out);
      upload({&po}, &out_dev, &out_cap, s);
      HIPCHK(issue(po, o.prec, o.B, s));
      for (Member* m : out)
        if (m->out_host)
          HIPCHK(hipMemcpyAsync(m->out, m->o_d, (size_t)m->W * m->H * m->C * sizeof(float),
                                hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (auto& r : leaving) complete(*r, r->m.get());
    }
    active.swap(next);
  }
}

extern "C" {

#define INPAINT_EXPORT __attribute__((visibility("default")))

INPAINT_EXPORT int inpaint_server_create(const inpaint_server_cfg* cfg, inpaint_server** srv) {
  return guarded([&] {
    if (!srv) fail(INPAINT_E_INVALID, "NULL server pointer");
    *srv = nullptr;
    if (cfg && cfg->struct_size != (int)sizeof(inpaint_server_cfg))
      fail(INPAINT_E_INVALID, "inpaint_server_cfg.struct_size must equal sizeof(inpaint_server_cfg)");
    std::unique_ptr<inpaint_server> sv(new inpaint_server());
    sv->o = resolve(cfg && cfg->opts.struct_size ? &cfg->opts : nullptr);
    sv->o.profile = 0;
    if (cg_schedule(sv->o.schedule))
      fail(INPAINT_E_INVALID, "the server runs the multigrid schedules (CG is a comparison schedule)");
    if (cfg && cfg->max_batch) sv->max_batch = cfg->max_batch;
    if (sv->max_batch < 1 || sv->max_batch > 1024) fail(INPAINT_E_INVALID, "max_batch must lie in [1, 1024]");
    HIPCHK(hipGetDevice(&sv->dev));
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    sv->budget = (cfg && cfg->hbm_budget) ? cfg->hbm_budget : fr / 10 * 8;
    HIPCHK(hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking));
    HIPCHK(hipMalloc(&sv->flags_dev, (size_t)sv->max_batch * kFlagInts * sizeof(int)));
    HIPCHK(hipHostMalloc(&sv->flags_host, (size_t)sv->max_batch * kFlagInts * sizeof(int), hipHostMallocDefault));
    for (int i = sv->max_batch - 1; i >= 0; --i) sv->free_slots.push_back(i);
    sv->t0 = std::chrono::steady_clock::now();
    sv->th = std::thread([p = sv.get()] { p->run(); });
    *srv = sv.release();
    return INPAINT_OK;
  });
}

INPAINT_EXPORT int inpaint_server_submit(inpaint_server* srv, const inpaint_problem* p, double tol,
                                         uint64_t* ticket) {
  return guarded([&] {
    if (!srv || !p || !ticket) fail(INPAINT_E_INVALID, "NULL pointer argument");
    validate_problem(*p, -1, srv->o);
    if (!(tol > 0.0 && tol < 1.0)) fail(INPAINT_E_INVALID, "tol must lie in (0, 1)");
    auto r = std::make_shared<Request>();
    r->p = *p;
    r->tol = tol;
    r->key = Key{srv->dev, p->W, p->H, p->channels, srv->o.B, srv->o.o, srv->o.B, srv->o.prec};
    {
      std::lock_guard<std::mutex> g(srv->mu);
      auto it = srv->ws_size.find(r->key);
      if (it == srv->ws_size.end()) it = srv->ws_size.emplace(r->key, workspace_bytes(r->key)).first;
      r->ws_bytes = it->second;
    }
    if (!is_device_ptr(p->f) || !is_device_ptr(p->mask) || !is_device_ptr(p->out))
      r->stage_bytes = staging_bytes(*p);
    if (r->ws_bytes + r->stage_bytes > srv->budget)
      fail(INPAINT_E_NOMEM, "the request's hierarchy exceeds the server's HBM budget");
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->broken) {
      g_err = srv->broken_msg;
      throw Fail{srv->broken};
    }
    if (srv->stop) fail(INPAINT_E_INVALID, "the server is shutting down");
    r->ticket = srv->next_ticket++;
    r->t_submit = srv->now_ms();
    srv->reqs[r->ticket] = r;
    srv->queue.push_back(r);
    *ticket = r->ticket;
    srv->cv_work.notify_one();
    return INPAINT_OK;
  });
}

static int collect(inpaint_server* srv, uint64_t ticket, inpaint_stats* st, bool block) {
  return guarded([&] {
    if (!srv) fail(INPAINT_E_INVALID, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) fail(INPAINT_E_INVALID, "unknown or already collected ticket");
    std::shared_ptr<Request> r = it->second;
    if (!r->done) {
      if (!block) return (int)INPAINT_PENDING;
      srv->cv_done.wait(lk, [&] { return r->done; });
    }
    if (st) *st = r->stats;
    srv->reqs.erase(ticket);
    if (r->status < 0) g_err = r->status == srv->broken ? srv->broken_msg : (r->m ? r->m->msg : "");
    return r->status;
  });
}

INPAINT_EXPORT int inpaint_server_poll(inpaint_server* srv, uint64_t ticket, inpaint_stats* st) {
  return collect(srv, ticket, st, false);
}

INPAINT_EXPORT int inpaint_server_wait(inpaint_server* srv, uint64_t ticket, inpaint_stats* st) {
  return collect(srv, ticket, st, true);
}

INPAINT_EXPORT void inpaint_server_destroy(inpaint_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  if (srv->th.joinable()) srv->th.join();
  int old = -1;
  (void)hipGetDevice(&old);
  (void)hipSetDevice(srv->dev);
  if (srv->s) (void)hipStreamSynchronize(srv->s);
  srv->pool.clear();
  if (srv->prep_dev) (void)hipFree(srv->prep_dev);
  if (srv->plan_dev) (void)hipFree(srv->plan_dev);
  if (srv->out_dev) (void)hipFree(srv->out_dev);
  if (srv->flags_dev) (void)hipFree(srv->flags_dev);
  if (srv->flags_host) (void)hipHostFree(srv->flags_host);
  if (srv->s) (void)hipStreamDestroy(srv->s);
  if (old >= 0) (void)hipSetDevice(old);
  delete srv;
}

}  // extern "C"
