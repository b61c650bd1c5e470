// The serving loop's device-independent core (see serve_core.h).
#include "serve_core.h"

#include <utility>

namespace inpaint {

ServeCore::ServeCore(std::unique_ptr<Executor> ex, int max_batch, size_t budget)
    : ex_(std::move(ex)), max_batch_(max_batch), budget_(budget) {
  for (int i = max_batch_ - 1; i >= 0; --i) free_slots_.push_back(i);
  t0_ = std::chrono::steady_clock::now();
  th_ = std::thread([this] { run(); });
}

ServeCore::~ServeCore() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
    cv_work_.notify_all();
  }
  if (th_.joinable()) th_.join();
  pool_.clear();
  ex_.reset();
}

double ServeCore::now_ms() const {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
}

// A hierarchy for r from the pool: an idle one of r's shape, else a new one
// after freeing idle hierarchies of other shapes as the budget requires; -1
// if r cannot fit now.
int ServeCore::take_hier(ServeRequest& r) {
  for (size_t i = 0; i < pool_.size(); ++i)
    if (!pool_busy_[i] && pool_[i] && pool_[i]->shape == r.shape) {
      const size_t extra = (r.stage_bytes && ex_->needs_staging(*pool_[i], r)) ? r.stage_bytes : 0;
      if (pool_bytes_ + extra > budget_ && !evict(extra, (int)i)) return -1;
      pool_bytes_ += extra;
      pool_busy_[i] = 1;
      return (int)i;
    }
  const size_t need = r.hier_bytes + r.stage_bytes;
  if (pool_bytes_ + need > budget_ && !evict(need, -1)) return -1;
  auto h = ex_->create(r);
  h->shape = r.shape;
  pool_bytes_ += need;
  for (size_t i = 0; i < pool_.size(); ++i)
    if (!pool_[i]) {
      pool_[i] = std::move(h);
      pool_busy_[i] = 1;
      return (int)i;
    }
  pool_.push_back(std::move(h));
  pool_busy_.push_back(1);
  return (int)pool_.size() - 1;
}

// Free idle hierarchies (not `keep`) until `need` more bytes fit the budget.
bool ServeCore::evict(size_t need, int keep) {
  for (size_t i = 0; i < pool_.size() && pool_bytes_ + need > budget_; ++i)
    if (pool_[i] && !pool_busy_[i] && (int)i != keep) {
      pool_bytes_ -= ex_->bytes(*pool_[i]);
      pool_[i].reset();
    }
  return pool_bytes_ + need <= budget_;
}

void ServeCore::complete(ServeRequest& r) {
  inpaint_stats st = r.stats;
  st.status = r.status;
  st.t_submit_ms = r.t_submit;
  st.t_start_ms = r.t_start;
  st.t_done_ms = now_ms();
  if (r.slot >= 0) free_slots_.push_back(r.slot);
  if (r.pool_idx >= 0) pool_busy_[r.pool_idx] = 0;
  r.slot = r.pool_idx = -1;
  ex_->release(r);
  std::lock_guard<std::mutex> g(mu_);
  r.stats = st;
  r.done = true;
  cv_done_.notify_all();
}

void ServeCore::run() {
  try {
    loop();
  } catch (const Fail& e) {
    std::lock_guard<std::mutex> g(mu_);
    broken_ = e.code;
    broken_msg_ = g_err;
  } catch (...) {
    std::lock_guard<std::mutex> g(mu_);
    broken_ = INPAINT_E_DEVICE;
    broken_msg_ = "unexpected exception in the server loop";
  }
  // fail whatever is left
  std::lock_guard<std::mutex> g(mu_);
  for (auto& kv : reqs_)
    if (!kv.second->done) {
      kv.second->status = broken_ ? broken_ : INPAINT_E_DEVICE;
      kv.second->stats.status = kv.second->status;
      kv.second->done = true;
    }
  queue_.clear();
  cv_done_.notify_all();
}

void ServeCore::loop() {
  ex_->start();
  std::vector<std::shared_ptr<ServeRequest>> active;  // prepared and cycling
  while (true) {
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_work_.wait(lk, [&] { return stop_ || !queue_.empty() || !active.empty(); });
      if (stop_ && queue_.empty() && active.empty()) return;
    }
    // 1. admission: arrival order, while a slot is free and the hierarchy fits
    std::vector<std::shared_ptr<ServeRequest>> fresh;
    while (active.size() + fresh.size() < (size_t)max_batch_) {
      std::shared_ptr<ServeRequest> r;
      {
        std::lock_guard<std::mutex> g(mu_);
        if (queue_.empty()) break;
        r = queue_.front();
      }
      const int idx = take_hier(*r);
      if (idx < 0) break;
      {
        std::lock_guard<std::mutex> g(mu_);
        queue_.pop_front();
      }
      r->pool_idx = idx;
      r->slot = free_slots_.back();
      free_slots_.pop_back();
      r->t_start = now_ms();
      fresh.push_back(r);
    }
    // 2. staging, coarse problems and input checks of the admitted requests
    std::vector<std::shared_ptr<ServeRequest>> cas;
    if (!fresh.empty()) {
      std::vector<ServeRequest*> fr;
      std::vector<ExecHier*> hs;
      for (auto& r : fresh) {
        fr.push_back(r.get());
        hs.push_back(pool_[r->pool_idx].get());
      }
      ex_->prepare(fr, hs);
      for (auto& r : fresh) {
        if (r->status < 0)
          complete(*r);
        else
          cas.push_back(r);
      }
    }
    // 3. one step for everybody: the cascade of the new requests, one V-cycle
    // of the running ones
    std::vector<ServeRequest*> c, g;
    for (auto& r : cas) c.push_back(r.get());
    for (auto& r : active) g.push_back(r.get());
    if (!c.empty() || !g.empty()) ex_->step(c, g);
    // 4. requests that are finished leave
    std::vector<std::shared_ptr<ServeRequest>> next, leaving;
    for (auto* list : {&cas, &active})
      for (auto& r : *list) (r->leaving ? leaving : next).push_back(r);
    if (!leaving.empty()) {
      std::vector<ServeRequest*> out;
      for (auto& r : leaving) out.push_back(r.get());
      ex_->finish(out);
      for (auto& r : leaving) complete(*r);
    }
    active.swap(next);
  }
}

uint64_t ServeCore::submit(const inpaint_problem& p, double tol) {
  auto r = std::make_shared<ServeRequest>();
  ex_->describe(p, &r->shape, &r->hier_bytes, &r->stage_bytes);
  if (!(tol > 0.0 && tol < 1.0)) fail(INPAINT_E_INVALID, "tol must lie in (0, 1)");
  if (r->hier_bytes + r->stage_bytes > budget_)
    fail(INPAINT_E_NOMEM, "the request's hierarchy exceeds the server's HBM budget");
  r->p = p;
  r->tol = tol;
  std::lock_guard<std::mutex> g(mu_);
  if (broken_) {
    g_err = broken_msg_;
    throw Fail{broken_};
  }
  if (stop_) fail(INPAINT_E_INVALID, "the server is shutting down");
  r->ticket = next_ticket_++;
  r->t_submit = now_ms();
  reqs_[r->ticket] = r;
  queue_.push_back(r);
  cv_work_.notify_one();
  return r->ticket;
}

int ServeCore::collect(uint64_t ticket, inpaint_stats* st, bool block) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = reqs_.find(ticket);
  if (it == reqs_.end()) fail(INPAINT_E_INVALID, "unknown or already collected ticket");
  std::shared_ptr<ServeRequest> r = it->second;
  if (!r->done) {
    if (!block) return INPAINT_PENDING;
    cv_done_.wait(lk, [&] { return r->done; });
  }
  if (st) *st = r->stats;
  reqs_.erase(ticket);
  if (r->status < 0) g_err = r->status == broken_ ? broken_msg_ : r->msg;
  return r->status;
}

}  // namespace inpaint
