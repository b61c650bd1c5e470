// Batched solve: n independent problems of any sizes advance together.  Every
// step of the method (the cascade and V-cycle of Section 4.2, the two halves of
// an ORAS iteration of Algorithm 2) becomes one launch over all problems that
// take part in it, problems in lockstep by level.  Each problem keeps its own
// workspace, norms and convergence flags and runs the same arithmetic in the
// same order as a solve of that problem alone, so its result is bit-identical.
// One V-cycle of the whole batch is captured once as a HIP graph and replayed
// until every problem has converged.
#include <hip/hip_runtime.h>

#include <array>
#include <list>
#include <map>

#include "batch.h"

namespace inpaint {
namespace {

// ---------------------------------------------------------------------------
// batch-only kernels
// ---------------------------------------------------------------------------

struct ResetArgs {
  int* active;
  int* status;
  int* checks;
  unsigned long long* cgstat;
  int C;
};

// Copy of one problem's flag block (kFlagInts ints: relres[4] doubles,
// active[4], status[4], checks[4] ints) into the batch's gathered array.
struct GatherArgs {
  const int* src;
  int* dst;
};

__global__ void __launch_bounds__(64) k_reset_b(const ResetArgs* __restrict__ args) {
  const ResetArgs a = args[blockIdx.x];
  const int t = threadIdx.x;
  if (t < a.C) a.active[t] = 1;
  if (t < 4) a.status[t] = 0;
  if (t < kKnownWords) a.status[kKnownAt + t] = 0;
  if (t < 4) a.checks[t] = 0;
  for (int i = t; i < 3 * a.C * kMaxLevels; i += blockDim.x) a.cgstat[i] = 0;
}

__global__ void __launch_bounds__(64) k_gather(const GatherArgs* __restrict__ args) {
  const GatherArgs a = args[blockIdx.x];
  const int t = threadIdx.x;
  if (t < kFlagInts) a.dst[t] = a.src[t];
}

}  // namespace

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------

void Plan::begin(int kind, int mode, int level) {
  open = Step{kind, mode, -1, level, 0, 0, 0, 0};
  pend.clear();
  pstart.assign(1, 0u);
}

void Plan::end() {
  if (open.n == 0) return;
  if (open.f32 < 0) open.f32 = 0;
  if (open.mode < 0) open.mode = 0;
  open.total = pstart.back();
  open.args = append(pend.data(), pend.size());
  open.start = append(pstart.data(), pstart.size() * sizeof(unsigned));
  steps.push_back(open);
  open.n = 0;
}

size_t Plan::append(const void* p, size_t n) {
  const size_t at = round_up(host.size(), 64);
  host.resize(at + n);
  std::memcpy(host.data() + at, p, n);
  return at;
}

void Plan::clear() {
  steps.clear();
  host.clear();
  delta.clear();
  cur0.clear();
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  exec = nullptr;
  graph = nullptr;
  dev = nullptr;
}

Plan::~Plan() { clear(); }

hipEvent_t Prof::event() {
  if (next == pool->size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    pool->push_back(e);
  }
  return (*pool)[next++];
}

namespace {

// inpaint_kernel class of a finest-grid launch, -1 for launches not timed
int kernel_class(const Step& st) {
  if (st.level != 0) return -1;
  switch (st.kind) {
    case S_STAGE: return INPAINT_K_STAGE;
    case S_RHS: return INPAINT_K_PYRAMID;
    case S_BLOCK: return INPAINT_K_BLOCK_SOLVE;
    case S_RESTRICT: return INPAINT_K_RESTRICT;
    case S_COARSE: return INPAINT_K_COARSE;
    case S_OUTPUT: return INPAINT_K_OUTPUT;
    case S_CG_DIR:
    case S_CG_STEP: return INPAINT_K_UPDATE;  // the CG schedule's iteration
    case S_PASS:
      switch (st.mode) {
        case PASS_RES: return INPAINT_K_RESIDUAL;
        case PASS_UPD:
        case PASS_UPD0:
        case PASS_FIN:
        case PASS_FIN0: return INPAINT_K_UPDATE;
        default: return INPAINT_K_PROLONG;  // PSOL, PCORR, PCORR0
      }
    default: return -1;
  }
}

hipError_t issue_step(const Step& st, const unsigned char* dev, int prec, int B, hipStream_t s);

}  // namespace

hipError_t issue(const Plan& P, int prec, int B, hipStream_t s, Prof* prof) {
  for (const Step& st : P.steps) {
    const int cls = prof ? kernel_class(st) : -1;
    if (cls < 0) {
      const hipError_t e = issue_step(st, P.dev, prec, B, s);
      if (e != hipSuccess) return e;
      continue;
    }
    hipEvent_t a = prof->event(), b = prof->event();
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = issue_step(st, P.dev, prec, B, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
    prof->recs.push_back({cls, a, b});
  }
  return hipSuccess;
}

namespace {

hipError_t issue_step(const Step& st, const unsigned char* dev, int prec, int B, hipStream_t s) {
  {
    const void* a = dev + st.args;
    const unsigned* start = (const unsigned*)(dev + st.start);
    hipError_t e = hipSuccess;
    switch (st.kind) {
      case S_RESET:
        hipLaunchKernelGGL(k_reset_b, dim3(st.n), dim3(64), 0, s, (const ResetArgs*)a);
        e = hipGetLastError();
        break;
      case S_GATHER:
        hipLaunchKernelGGL(k_gather, dim3(st.n), dim3(64), 0, s, (const GatherArgs*)a);
        e = hipGetLastError();
        break;
      case S_STAGE: e = launch_stage_b((const StageArgs*)a, start, st.n, st.total, s); break;
      case S_RHS:
        e = launch_rhs_b((const RhsArgs*)a, start, st.n, st.total, prec, st.f32, s);
        break;
      case S_PASS:
        e = launch_pass_b(st.mode, (const PassArgs*)a, start, st.n, st.total, prec, st.f32, s);
        break;
      case S_RESTRICT:
        e = launch_restrict_b((const RestrictArgs*)a, start, st.n, st.total, prec, st.f32, s);
        break;
      case S_BLOCK:
        e = launch_block_b((const BlockArgs*)a, start, st.n, st.total, prec, st.f32, B, s);
        break;
      case S_COARSE:
        e = launch_coarse_b((const CoarseArgs*)a, start, st.n, st.total, prec, st.f32, B, s);
        break;
      case S_OUTPUT: e = launch_output_b((const OutputArgs*)a, start, st.n, st.total, s); break;
      case S_CG_DIR: e = launch_cg_dir_b((const CgArgs*)a, start, st.n, st.total, s); break;
      case S_CG_STEP: e = launch_cg_step_b((const CgArgs*)a, start, st.n, st.total, s); break;
      case S_WARM: e = launch_warm_b((const WarmArgs*)a, start, st.n, st.total, s); break;
      default: e = hipErrorInvalidValue;
    }
    return e;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// plan builders: each walks the members in lockstep and calls their Run's
// argument builders in the order a solve of that member alone would launch
// ---------------------------------------------------------------------------

namespace {

template <class Pred>
std::vector<Member*> subset(const std::vector<Member*>& ms, Pred pred) {
  std::vector<Member*> r;
  for (Member* m : ms)
    if (pred(m)) r.push_back(m);
  return r;
}

int max_coarsest(const std::vector<Member*>& ms) {
  int v = 0;
  for (const Member* m : ms) v = std::max(v, m->Lc());
  return v;
}

bool corr0(const Member* m) { return m->R->corr0(); }

void step_block(Plan& P, const std::vector<Member*>& ms, int l) {
  P.begin(S_BLOCK, 0, l);
  for (Member* m : ms) {
    const BlockArgs a = m->R->make_block(l);
    P.add(a, work_block(a, m->C), a.level0);
  }
  P.end();
}

// The precision form's last update of a cycle on the finest grid (see
// Run::make_final).
void step_final(Plan& P, const std::vector<Member*>& ms, bool blocks) {
  P.begin(S_PASS, -1, 0);
  for (Member* m : ms) {
    const PassArgs a = m->R->make_final(true, blocks);
    P.add_pass(a, work_pass(a, m->C));
  }
  P.end();
}

// One ORAS iteration on level l of every member in ms (need: a later launch
// reads the norm its update writes).
// One ORAS iteration on level l.  defer: its new iterate is read only by the
// next prolongation from level l, which adds the block corrections itself
// (no update pass).
void step_oras(Plan& P, const std::vector<Member*>& ms, int l, bool check, bool rest,
               bool need = true, bool defer = false) {
  step_block(P, ms, l);
  if (defer) {
    for (Member* m : ms) m->R->defer_update(l);
    return;
  }
  P.begin(S_PASS, -1, l);
  for (Member* m : ms) {
    const PassArgs a = m->R->make_update(l, check, rest, need);
    P.add_pass(a, work_pass(a, m->C));
  }
  P.end();
}

// One ORAS iteration on the finest grid ending in the convergence test: in
// the precision form its update is the final update of the correction.
void step_oras_checked(Plan& P, const std::vector<Member*>& ms) {
  const auto corr = subset(ms, corr0);
  const auto plain = subset(ms, [](Member* m) { return !corr0(m); });
  if (!plain.empty()) step_oras(P, plain, 0, true, false);
  if (!corr.empty()) {
    step_block(P, corr, 0);
    step_final(P, corr, true);
  }
}

void step_residual(Plan& P, const std::vector<Member*>& ms) {
  P.begin(S_PASS, -1, 0);
  for (Member* m : ms) {
    const PassArgs a = m->R->make_residual(0, true);
    P.add_pass(a, work_pass(a, m->C));
  }
  P.end();
}

// A V-cycle on level l0 of every member (Section 4.2): the members' down
// sweeps run level by level, the coarsest-grid solves of all members in one
// launch (two when some member has a single level), then the up sweeps.
void build_vcycle(Plan& P, const std::vector<Member*>& ms, int l0, const Opts& o) {
  const int maxLc = max_coarsest(ms);
  for (int l = l0; l < maxLc; ++l) {
    const auto part = subset(ms, [&](Member* m) { return l < m->Lc(); });
    for (int i = 0; i < o.pre; ++i) step_oras(P, part, l, false, i == o.pre - 1);
    if (o.pre == 0) {
      P.begin(S_RESTRICT, 0, l);
      for (Member* m : part) {
        const RestrictArgs a = m->R->make_restrict(l);
        P.add(a, work_restrict(a, m->C), a.level0);
      }
      P.end();
    }
  }
  P.begin(S_COARSE, 0, maxLc);
  for (Member* m : ms)
    if (m->Lc() > 0) {
      const CoarseArgs a = m->R->make_coarse(m->Lc(), true);
      P.add(a, work_coarse(a, m->C), a.level0);
    }
  P.end();
  const auto flat = subset(ms, [](Member* m) { return m->Lc() == 0; });
  P.begin(S_COARSE, 0, 0);
  for (Member* m : flat) {
    const CoarseArgs a = m->R->make_coarse(0, false);
    P.add(a, work_coarse(a, m->C), a.level0);
  }
  P.end();
  step_residual(P, flat);
  for (int l = maxLc - 1; l >= l0; --l) {
    const auto part = subset(ms, [&](Member* m) { return l < m->Lc(); });
    const auto corr = subset(part, [&](Member* m) { return l == 0 && corr0(m); });
    const auto plain = subset(part, [&](Member* m) { return !(l == 0 && corr0(m)); });
    P.begin(S_PASS, -1, l);
    for (Member* m : plain) {
      const PassArgs a = m->R->make_prolong(l, PASS_PCORR, l == 0 && o.post == 0, o.post > 0);
      P.add_pass(a, work_pass(a, m->C));
    }
    P.end();
    // on coarser levels the last post-smoothing's norm is not read, and its
    // update is left to the next prolongation
    for (int i = 0; i < o.post; ++i)
      step_oras(P, plain, l, l == 0 && i == o.post - 1, false, l == 0 || i + 1 < o.post,
                l > 0 && i + 1 == o.post);
    if (corr.empty()) continue;
    // precision form: the correction e of the float32 iterate gets the coarse
    // correction and the post-smoothing; the last update adds e to u and tests
    P.begin(S_PASS, -1, 0);
    for (Member* m : corr) {
      const PassArgs a = m->R->make_prolong(0, PASS_PCORR, false, o.post > 0);
      P.add_pass(a, work_pass(a, m->C));
    }
    P.end();
    for (int i = 0; i + 1 < o.post; ++i) step_oras(P, corr, 0, false, false);
    if (o.post > 0) step_block(P, corr, 0);
    step_final(P, corr, o.post > 0);
  }
}

}  // namespace

// Plain CG (comparison schedules): the true residual of level l (with the
// convergence test on the finest grid), and iterations of the direction and
// step passes.
void step_cg_residual(Plan& P, const std::vector<Member*>& ms, int l = 0, bool check = true) {
  P.begin(S_PASS, -1, l);
  for (Member* m : ms) {
    const PassArgs a = m->R->make_cg_residual(l, check);
    P.add_pass(a, work_pass(a, m->C));
  }
  P.end();
}

void step_cg(Plan& P, const std::vector<Member*>& ms, bool first, int l = 0) {
  P.begin(S_CG_DIR, 0, l);
  for (Member* m : ms) {
    const CgArgs a = m->R->make_cg_dir(l, first);
    P.add(a, work_cg(a, m->C));
  }
  P.end();
  P.begin(S_CG_STEP, 0, l);
  for (Member* m : ms) {
    const CgArgs a = m->R->make_cg_step(l);
    P.add(a, work_cg(a, m->C));
  }
  P.end();
}

// n CG iterations on level l, restarted from the residual the previous pass
// left there (the problem changed: a prolongation or a restriction).
void smooth_cg(Plan& P, const std::vector<Member*>& ms, int l, int n) {
  for (int i = 0; i < n; ++i) step_cg(P, ms, i == 0, l);
}

// A prolongation to level l of every member in ms whose residual norm starts
// the CG smoothing of level l.
void step_cg_prolong(Plan& P, const std::vector<Member*>& ms, int l, int mode, bool check) {
  P.begin(S_PASS, -1, l);
  for (Member* m : ms) {
    const PassArgs a = m->R->make_cg_prolong(l, mode, check);
    P.add_pass(a, work_pass(a, m->C));
  }
  P.end();
}

constexpr int kCgPerCycle = 8;

// The multigrid CG counterpart's V-cycle: the ORAS V-cycle's structure with
// CG as pre- and post-smoother on every level; the residual after
// pre-smoothing is evaluated in float64 and restricted by the plain
// restriction.
void build_vcycle_cg(Plan& P, const std::vector<Member*>& ms, const Opts& o) {
  const int maxLc = max_coarsest(ms);
  for (int l = 0; l < maxLc; ++l) {
    const auto part = subset(ms, [&](Member* m) { return l < m->Lc(); });
    smooth_cg(P, part, l, o.pre);
    P.begin(S_PASS, -1, l);
    for (Member* m : part) {
      const PassArgs a = m->R->make_cg_pre_residual(l);
      P.add_pass(a, work_pass(a, m->C));
    }
    P.end();
    P.begin(S_RESTRICT, 0, l);
    for (Member* m : part) {
      const RestrictArgs a = m->R->make_cg_restrict(l);
      P.add(a, work_restrict(a, m->C), a.level0);
    }
    P.end();
  }
  P.begin(S_COARSE, 0, maxLc);
  for (Member* m : ms)
    if (m->Lc() > 0) {
      const CoarseArgs a = m->R->make_coarse(m->Lc(), true);
      P.add(a, work_coarse(a, m->C), a.level0);
    }
  P.end();
  const auto flat = subset(ms, [](Member* m) { return m->Lc() == 0; });
  P.begin(S_COARSE, 0, 0);
  for (Member* m : flat) {
    const CoarseArgs a = m->R->make_coarse(0, false);
    P.add(a, work_coarse(a, m->C), a.level0);
  }
  P.end();
  step_cg_residual(P, flat);
  for (int l = maxLc - 1; l >= 0; --l) {
    const auto part = subset(ms, [&](Member* m) { return l < m->Lc(); });
    step_cg_prolong(P, part, l, PASS_PCORR, l == 0 && o.post == 0);
    smooth_cg(P, part, l, o.post);
    if (l == 0 && o.post > 0) step_cg_residual(P, part);
  }
}

// The coarse-to-fine initial guess (Section 4.2) of every member.
void build_cascade(Plan& P, const std::vector<Member*>& ms, const Opts& o) {
  if (o.schedule == INPAINT_SCHED_WARM) {
    // no cascade: the residual of the guess and the first convergence test
    step_residual(P, ms);
    return;
  }
  if (o.schedule == INPAINT_SCHED_CG) {
    step_cg_residual(P, ms);
    step_cg(P, ms, true);
    return;
  }
  if (o.schedule == INPAINT_SCHED_SINGLE) {
    step_residual(P, ms);
    return;
  }
  const bool cg = cg_schedule(o.schedule);
  const auto flat = subset(ms, [](Member* m) { return m->Lc() == 0; });
  if (cg)
    step_cg_residual(P, flat);
  else
    step_residual(P, flat);
  const auto deep = subset(ms, [](Member* m) { return m->Lc() > 0; });
  P.begin(S_COARSE, 0, max_coarsest(deep));
  for (Member* m : deep) {
    m->R->top = m->Lc();
    const CoarseArgs a = m->R->make_coarse(m->Lc(), true);
    P.add(a, work_coarse(a, m->C), a.level0);
  }
  P.end();
  for (int l = max_coarsest(deep) - 1; l >= 0; --l) {
    const auto part = subset(deep, [&](Member* m) { return l < m->Lc(); });
    for (Member* m : part) m->R->top = l;
    if (cg) {
      step_cg_prolong(P, part, l, PASS_PSOL, l == 0);
      if (l == 0) break;
      smooth_cg(P, part, l, o.pre);
      continue;
    }
    P.begin(S_PASS, -1, l);
    for (Member* m : part) {
      const PassArgs a = m->R->make_prolong(l, PASS_PSOL, l == 0);
      P.add_pass(a, work_pass(a, m->C));
    }
    P.end();
    if (l == 0) break;
    if (o.schedule == INPAINT_SCHED_FMG)
      build_vcycle(P, part, l, o);
    else
      step_oras(P, part, l, false, false, false, true);
  }
  // the multilevel CG counterpart continues with plain CG on the finest grid
  if (o.schedule == INPAINT_SCHED_CG_MULTILEVEL) step_cg(P, ms, true);
}

void build_cycle(Plan& P, const std::vector<Member*>& ms, const Opts& o) {
  if (o.schedule == INPAINT_SCHED_RFMG || o.schedule == INPAINT_SCHED_FMG ||
      o.schedule == INPAINT_SCHED_WARM) {
    build_vcycle(P, ms, 0, o);
  } else if (o.schedule == INPAINT_SCHED_CG_MULTIGRID) {
    build_vcycle_cg(P, ms, o);
  } else if (cg_schedule(o.schedule)) {
    for (int i = 0; i < kCgPerCycle; ++i) step_cg(P, ms, false);
    step_cg_residual(P, ms);
  } else {
    step_oras_checked(P, ms);
  }
}

void add_gather(Plan& P, const std::vector<Member*>& ms, int* flags_dev) {
  if (!flags_dev) return;  // a batch of one polls its own flag block
  P.begin(S_GATHER);
  for (Member* m : ms) P.add(GatherArgs{(const int*)m->ws->relres, flags_dev + kFlagInts * m->slot}, 1u);
  P.end();
}

std::vector<int> level_state(const std::vector<Member*>& ms) {
  std::vector<int> s;
  for (Member* m : ms) {
    for (int l = 0; l < m->ws->L; ++l) s.push_back(m->ws->lv[l].cur);
    s.push_back(m->ws->lv[0].ecur);
    s.push_back(m->ws->lv[0].ezero);
    s.push_back(m->R->cg_slot);
    s.push_back(m->R->cg_p);
  }
  return s;
}

// ---------------------------------------------------------------------------
// batch contexts (device copies of the plans, graphs, flag buffers), cached by
// the workspaces, options and tolerance of a batch
// ---------------------------------------------------------------------------

BatchCtx::~BatchCtx() {
  int old = -1;
  (void)hipGetDevice(&old);
  (void)hipSetDevice(dev_id);
  cascade.clear();
  for (Plan& p : cycle) p.clear();
  if (plan_dev) (void)hipFree(plan_dev);
  if (call_dev) (void)hipFree(call_dev);
  if (flags_dev) (void)hipFree(flags_dev);
  if (flags_host) (void)hipHostFree(flags_host);
  if (cap) (void)hipStreamDestroy(cap);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (old >= 0) (void)hipSetDevice(old);
}

namespace {

std::mutex g_bmu;
std::list<std::shared_ptr<BatchCtx>> g_bcache;  // most recently used first
constexpr size_t kBatchCacheSize = 32;

std::string ctx_key(int dev, const std::vector<Member*>& ms, const Opts& o, double tol) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
  put(&dev, sizeof dev);
  put(&o, sizeof o);
  put(&tol, sizeof tol);
  // workspace serials, never reused: a plan cached for a workspace that has
  // since been freed can never match again
  for (const Member* m : ms) put(&m->ws->serial, sizeof m->ws->serial);
  return k;
}

std::shared_ptr<BatchCtx> batch_ctx(int dev, const std::vector<Member*>& ms, const Opts& o,
                                    double tol, int n) {
  const std::string key = ctx_key(dev, ms, o, tol);
  {
    std::lock_guard<std::mutex> g(g_bmu);
    for (auto it = g_bcache.begin(); it != g_bcache.end(); ++it)
      if ((*it)->key == key) {
        auto c = *it;
        g_bcache.erase(it);
        g_bcache.push_front(c);
        return c;
      }
  }
  auto c = std::make_shared<BatchCtx>();
  c->key = key;
  c->dev_id = dev;
  c->n = n;
  HIPCHK(hipMalloc(&c->flags_dev, (size_t)n * kFlagInts * sizeof(int)));
  HIPCHK(hipHostMalloc(&c->flags_host, (size_t)n * kFlagInts * sizeof(int), hipHostMallocDefault));
  HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIPCHK(hipEventCreate(&c->ev0));
  HIPCHK(hipEventCreate(&c->ev1));
  std::lock_guard<std::mutex> g(g_bmu);
  g_bcache.push_front(c);
  while (g_bcache.size() > kBatchCacheSize) g_bcache.pop_back();
  return c;
}

}  // namespace

void upload(std::vector<Plan*> plans, unsigned char** buf, size_t* cap, hipStream_t s) {
  size_t need = 0;
  for (Plan* p : plans) need += round_up(p->host.size(), 256);
  if (need > *cap) {
    if (*buf) {
      HIPCHK(hipStreamSynchronize(s));
      HIPCHK(hipFree(*buf));
      *buf = nullptr;
      *cap = 0;
    }
    HIPCHK(hipMalloc(buf, need));
    *cap = need;
  }
  size_t off = 0;
  for (Plan* p : plans) {
    p->dev = *buf + off;
    if (!p->host.empty())
      HIPCHK(hipMemcpyAsync(p->dev, p->host.data(), p->host.size(), hipMemcpyHostToDevice, s));
    off += round_up(p->host.size(), 256);
  }
}

namespace {

void capture(Plan& P, BatchCtx& c, int prec, int B) {
  HIPCHK(hipStreamBeginCapture(c.cap, hipStreamCaptureModeThreadLocal));
  const hipError_t e = issue(P, prec, B, c.cap);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c.cap, &g);
  HIPCHK(e);
  HIPCHK(e2);
  P.graph = g;
  HIPCHK(hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0));
}

void run_plan(const Plan& P, int prec, int B, hipStream_t s) {
  if (P.exec)
    HIPCHK(hipGraphLaunch(P.exec, s));
  else
    HIPCHK(issue(P, prec, B, s));
}

}  // namespace

bool apply_flags(const int* flags_host, const std::vector<Member*>& ms, const Plan& P) {
  bool all = true;
  for (size_t i = 0; i < ms.size(); ++i) {
    Member* m = ms[i];
    const int* blk = flags_host + kFlagInts * m->slot;
    const double* rr = (const double*)blk;
    const int* act = blk + 8;
    const int* st = blk + 12;
    if (st[0] & 4) fail(INPAINT_E_DEVICE, "a norm partial never arrived (spin budget exhausted)");
    if (m->done) continue;
    bool d = true;
    for (int ch = 0; ch < m->C; ++ch) {
      if (m->final_cur[ch] < 0) {
        m->rel[ch] = rr[ch];
        if (!act[ch] || !std::isfinite(rr[ch])) m->final_cur[ch] = P.cur0[i];
      }
      d = d && m->final_cur[ch] >= 0;
    }
    m->done = d;
    all = all && d;
  }
  return all;
}

void account(const std::vector<Member*>& ms, const Plan& P) {
  for (size_t i = 0; i < ms.size(); ++i) {
    Member* m = ms[i];
    if (m->done) continue;
    m->oras += P.delta[i][0];
    m->blocks += P.delta[i][1];
    m->finest_blocks += P.delta[i][2];
  }
}

void finish_member(Member* m, int last_cur0) {
  bool diverged = false;
  for (int ch = 0; ch < m->C; ++ch) {
    if (m->final_cur[ch] < 0) m->final_cur[ch] = last_cur0;
    if (!std::isfinite(m->rel[ch])) diverged = true;
  }
  if (diverged) {
    m->status = INPAINT_E_DIVERGED;
    m->msg = "the residual became non-finite";
  } else if (!m->done) {
    m->status = INPAINT_NOT_CONVERGED;
    m->msg = "cycle cap reached before the tolerance";
  }
}

bool apply_counted(const int* flags_host, const std::vector<Member*>& ms,
                   const std::vector<const Plan*>& seq) {
  bool all = true;
  for (size_t i = 0; i < ms.size(); ++i) {
    Member* m = ms[i];
    const int* blk = flags_host + kFlagInts * m->slot;
    const double* rr = (const double*)blk;
    const int* act = blk + 8;
    const int* st = blk + 12;
    const int* tests = blk + 16;
    if (st[0] & 4) fail(INPAINT_E_DEVICE, "a norm partial never arrived (spin budget exhausted)");
    bool d = true;
    int last = 0;  // index in seq of the last plan that iterated the member
    for (int ch = 0; ch < m->C; ++ch) {
      // one test per plan while the channel iterates: a channel that stopped
      // (converged, or a non-finite residual) stopped in plan tests - 1
      const int k = tests[ch];
      if (k < 1 || k > (int)seq.size()) fail(INPAINT_E_DEVICE, "inconsistent convergence-test count");
      m->rel[ch] = rr[ch];
      if (!act[ch] || !std::isfinite(rr[ch])) {
        m->final_cur[ch] = seq[k - 1]->cur0[i];
        last = std::max(last, k - 1);
      } else {
        m->final_cur[ch] = -1;
        d = false;
      }
    }
    if (!d) last = (int)seq.size() - 1;
    m->done = d;
    m->cycles = last;
    m->oras = m->blocks = m->finest_blocks = 0;
    for (int p = 0; p <= last; ++p) {
      m->oras += seq[p]->delta[i][0];
      m->blocks += seq[p]->delta[i][1];
      m->finest_blocks += seq[p]->delta[i][2];
    }
    all = all && d;
  }
  return all;
}

void reset_member(Member* m) {
  m->status = INPAINT_OK;
  m->msg.clear();
  m->final_cur.assign(m->C, -1);
  m->rel.assign(m->C, 0.0);
  m->cycles = 0;
  m->done = false;
  m->oras = m->blocks = m->finest_blocks = 0;
}

void fill_stats(const Member* m, inpaint_stats& st) {
  std::memset(&st, 0, sizeof st);
  st.status = m->status;
  st.levels = m->ws ? m->ws->L : 0;
  if (m->status == INPAINT_OK || m->status == INPAINT_NOT_CONVERGED ||
      m->status == INPAINT_E_DIVERGED) {
    double r = 0.0;
    for (int ch = 0; ch < m->C; ++ch) r = std::max(r, m->rel[ch]);
    st.rel_res = m->status == INPAINT_E_DIVERGED ? NAN : r;
    st.cycles = m->cycles;
    st.oras_iters = (int)(m->oras * m->C);
    st.finest_block_solves = m->finest_blocks;
  }
}

// Reads the flag block written by the prepare plan: input checks of f and the mask.
void check_prepared(const int* flags_host, Member* m) {
  const int st = input_checks(flags_host + kFlagInts * m->slot + 12);
  if (st & 1) {
    m->status = INPAINT_E_INVALID;
    m->msg = "f is not finite at a known pixel";
  } else if (!(st & 2)) {
    m->status = INPAINT_E_EMPTY_MASK;
    m->msg = "mask has no known pixel: the system is singular";
  }
}

void validate_problem(const inpaint_problem& p, int i, const Opts& o) {
  try {
    check_dims(p.f, p.mask, p.W, p.H, p.channels);
    check_geometry(p.W, p.H, o.B, o.o);
    if (!p.out) fail(INPAINT_E_INVALID, "NULL pointer argument");
    const size_t nf = (size_t)p.W * p.H * p.channels * sizeof(float);
    if (p.out != p.f && overlap(p.out, nf, p.f, nf)) fail(INPAINT_E_INVALID, "out partially overlaps f");
    if (overlap(p.out, nf, p.mask, (size_t)p.W * p.H)) fail(INPAINT_E_INVALID, "out overlaps mask");
  } catch (const Fail&) {
    if (i >= 0) g_err = "problem " + std::to_string(i) + ": " + g_err;
    throw;
  }
}

// ---------------------------------------------------------------------------
// the batched solve
// ---------------------------------------------------------------------------

void init_member(Member& m, const inpaint_problem& p, Workspace* ws, const Opts& o, double tol,
                 hipStream_t s) {
  m.W = p.W;
  m.H = p.H;
  m.C = p.channels;
  m.ws = ws;
  m.R.reset(new Run{m.ws, o, s, m.C, tol});
  const bool fd = is_device_ptr(p.f), md = is_device_ptr(p.mask), od = is_device_ptr(p.out);
  if (!fd || !md || !od) ensure_staging(m.ws);
  if (cg_schedule(o.schedule)) ensure_cg(m.ws);
  const size_t nf = (size_t)m.W * m.H * m.C * sizeof(float);
  m.f_d = p.f;
  m.m_d = p.mask;
  m.o_d = p.out;
  m.out_host = !od;
  m.out = p.out;
  if (!fd) {
    HIPCHK(hipMemcpyAsync(m.ws->f_dev, p.f, nf, hipMemcpyHostToDevice, s));
    m.f_d = m.ws->f_dev;
  }
  if (!md) {
    HIPCHK(hipMemcpyAsync(m.ws->m_dev, p.mask, (size_t)m.W * m.H, hipMemcpyHostToDevice, s));
    m.m_d = m.ws->m_dev;
  }
  if (!od) {
    m.o_d = m.ws->o_dev;
    // a warm start reads its guess from out
    if (o.schedule == INPAINT_SCHED_WARM)
      HIPCHK(hipMemcpyAsync(m.o_d, p.out, nf, hipMemcpyHostToDevice, s));
  }
  m.final_cur.assign(m.C, -1);
  m.rel.assign(m.C, 0.0);
}

// Prepare plan: reset flags, stage every member's (f, mask) into level 0 with
// its reference residual, build the coarse masks and known values level by
// level, gather the flags (the input checks).
void build_prepare(Plan& P, const std::vector<Member*>& ms, const Opts& o, int* flags_dev) {
  // single-level schedules need no pyramid and start from u = C f
  const bool single = o.schedule == INPAINT_SCHED_SINGLE || o.schedule == INPAINT_SCHED_CG;
  P.begin(S_RESET);
  for (Member* m : ms) P.add(ResetArgs{m->ws->active, m->ws->status, m->ws->checks, m->ws->cgstat, m->C}, 1u);
  P.end();
  P.begin(S_STAGE, 0, 0);
  for (Member* m : ms) {
    Workspace* ws = m->ws;
    Level& L0 = ws->lv[0];
    L0.cur = 0;
    L0.ecur = 0;
    L0.ezero = true;
    NormOut den = m->R->norm(0, false);
    den.mode = NORM_FULL;
    den.out = ws->den;
    den.rho = ws->rho;
    den.inv_n = 1.0 / ((double)m->W * (double)m->H);
    const StageArgs a{m->f_d, m->m_d, m->W, m->H, m->W, m->C, L0.v, L0.c, L0.b,
                      (single || ws->L == 1) ? L0.u[0] : nullptr, ws->status, den};
    P.add(a, work_stage(a));
  }
  P.end();
  if (o.schedule == INPAINT_SCHED_WARM) {
    // the caller's guess (in out) becomes the finest iterate, known pixels b
    P.begin(S_WARM, 0, 0);
    for (Member* m : ms) {
      const Level& L0 = m->ws->lv[0];
      const WarmArgs a{L0.v, L0.c, L0.b, L0.u[0], m->o_d, m->W, m->C};
      P.add(a, work_warm(a));
    }
    P.end();
  }
  if (!single) {
    int maxL = 0;
    for (Member* m : ms) maxL = std::max(maxL, m->ws->L);
    for (int l = 0; l + 1 < maxL; ++l) {
      const auto part = subset(ms, [&](Member* m) { return l + 1 < m->ws->L; });
      P.begin(S_RHS, 0, l);
      for (Member* m : part) {
        Level& F = m->ws->lv[l];
        Level& Cl = m->ws->lv[l + 1];
        Cl.cur = 0;
        const RhsArgs a{F.v, Cl.v, F.c, F.b, Cl.c, Cl.b, m->C, o.rhs == INPAINT_RHS_NAIVE ? 1 : 0};
        P.add(a, work_rhs(a), l == 0 ? 1 : 0);
      }
      P.end();
    }
  }
  add_gather(P, ms, flags_dev);
}

void build_output(Plan& P, const std::vector<Member*>& ms) {
  P.begin(S_OUTPUT, 0, 0);
  for (Member* m : ms) {
    const Level& L0 = m->ws->lv[0];
    OutputArgs a{};
    a.lv = L0.v;
    a.c = L0.c;
    a.b = L0.b;
    for (int ch = 0; ch < kMaxChannels; ++ch) a.u[ch] = L0.u[m->final_cur[ch < m->C ? ch : 0]];
    a.out = m->o_d;
    a.Pout = m->W;
    a.C = m->C;
    a.den = m->ws->den;
    P.add(a, work_output(a));
  }
  P.end();
}

// The output issued right after the V-cycles the last solve in context c
// needed, before their convergence tests are read back: each channel's final
// buffer is chosen on the device from its test count (nplan plans issued: the
// cascade and the cycles), and a channel that has not stopped is left to the
// host-selected output that follows more cycles.
static void build_output_selected(Plan& P, const std::vector<Member*>& ms, const BatchCtx& c,
                                  int nplan) {
  P.begin(S_OUTPUT, 0, 0);
  for (size_t i = 0; i < ms.size(); ++i) {
    const Member* m = ms[i];
    const Level& L0 = m->ws->lv[0];
    OutputArgs a{};
    a.lv = L0.v;
    a.c = L0.c;
    a.b = L0.b;
    a.u[0] = L0.u[0];
    a.u[1] = L0.u[1];
    a.out = m->o_d;
    a.Pout = m->W;
    a.C = m->C;
    a.den = m->ws->den;
    a.flags = (const int*)m->ws->relres;
    a.nplan = nplan;
    a.ncycle = c.ncycle;
    a.cur[0] = c.cascade.cur0[i];
    a.cur[1] = c.cycle[0].cur0[i];
    a.cur[2] = c.cycle[c.ncycle > 1 ? 1 : 0].cur0[i];
    P.add(a, work_output(a));
  }
  P.end();
}

int solve_batched_impl(const inpaint_problem* probs, int n, double tol, const inpaint_opts* opts,
                       void* stream, inpaint_stats* stats) {
  if (!probs) fail(INPAINT_E_INVALID, "NULL problem array");
  if (n < 1) fail(INPAINT_E_INVALID, "n must be >= 1");
  if (!(tol > 0.0 && tol < 1.0)) fail(INPAINT_E_INVALID, "tol must lie in (0, 1)");
  Opts o = resolve(opts);
  o.profile = 0;
  for (int i = 0; i < n; ++i) validate_problem(probs[i], i, o);
  {
    std::vector<std::pair<const char*, const char*>> spans;
    for (int i = 0; i < n; ++i) {
      const char* a = (const char*)probs[i].out;
      spans.push_back({a, a + (size_t)probs[i].W * probs[i].H * probs[i].channels * sizeof(float)});
    }
    std::sort(spans.begin(), spans.end());
    for (int i = 1; i < n; ++i)
      if (spans[i].first < spans[i - 1].second)
        fail(INPAINT_E_INVALID, "the outputs of two problems overlap");
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<std::unique_ptr<Member>> own;
  std::vector<Member*> all;
  for (int i = 0; i < n; ++i) {
    own.emplace_back(new Member());
    Member& m = *own.back();
    m.idx = m.slot = i;
    acquire(m.lease, probs[i].W, probs[i].H, probs[i].channels, o.B, o.o, coarsest_side(o.B), o.prec);
    init_member(m, probs[i], m.lease.ws, o, tol, s);
    all.push_back(own.back().get());
  }
  const float ms = run_batch(all, o, tol, s, nullptr);
  int ret = INPAINT_OK;
  std::string msg;
  for (Member* m : all) {
    if (ret == INPAINT_OK || (ret == INPAINT_NOT_CONVERGED && m->status < 0)) {
      if (m->status != INPAINT_OK) {
        ret = m->status;
        msg = "problem " + std::to_string(m->idx) + ": " + m->msg;
      }
    }
    if (stats) {
      fill_stats(m, stats[m->idx]);
      stats[m->idx].gpu_ms = ms;
    }
  }
  g_err = msg;
  return ret;
}

float run_batch(const std::vector<Member*>& all, const Opts& o, double tol, hipStream_t s,
                Prof* prof) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const int n = (int)all.size();
  auto ctx = batch_ctx(dev, all, o, tol, n);
  BatchCtx& c = *ctx;
  const int prec = o.prec, B = o.B;

  // prepare: staging and hierarchies; members whose data is rejected leave
  HIPCHK(hipEventRecord(c.ev0, s));
  Plan prep;
  // A batch of one reads its workspace's flag block directly: no gather launches.
  int* const gather_to = n == 1 ? nullptr : c.flags_dev;
  const void* const flags_src = n == 1 ? (const void*)all[0]->ws->relres : (const void*)c.flags_dev;
  build(prep, all, [&] { build_prepare(prep, all, o, gather_to); });
  // With plans cached for every member and the cycle count of the last solve
  // in this context, the solve runs ahead: the input checks and the first
  // convergence tests are read back once, after that many V-cycles (a channel
  // that converges earlier skips the remaining launches) and the output
  // (device-selected: when every channel has stopped by then, the results
  // are in place when the tests are read).
  const std::string all_live(n, 1);
  const bool ahead = !prof && c.expect > 0 && c.live_key == all_live;
  const int nahead = ahead ? std::min(c.expect, o.max_cycles) : 0;
  Plan spec;
  if (ahead) {
    build_output_selected(spec, all, c, 1 + nahead);
    upload({&prep, &spec}, &c.call_dev, &c.call_cap, s);
  } else {
    upload({&prep}, &c.call_dev, &c.call_cap, s);
  }
  HIPCHK(issue(prep, prec, B, s, prof));
  std::vector<Member*> live;
  std::string live_key;
  bool written = false;
  if (ahead) {
    live = all;
    live_key = all_live;
  } else {
    HIPCHK(hipMemcpyAsync(c.flags_host, flags_src, (size_t)n * kFlagInts * sizeof(int),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (Member* m : all) {
      check_prepared(c.flags_host, m);
      live_key.push_back(m->status == INPAINT_OK ? 1 : 0);
      if (m->status == INPAINT_OK) live.push_back(m);
    }
  }

  if (!live.empty()) {
    // cascade and cycle plans, built once per batch context
    if (c.live_key != live_key) {
      c.cascade.clear();
      for (Plan& p : c.cycle) p.clear();
      c.live_key = live_key;
      build(c.cascade, live, [&] {
        build_cascade(c.cascade, live, o);
        add_gather(c.cascade, live, gather_to);
      });
      const std::vector<int> s0 = level_state(live);
      c.ncycle = 0;
      for (int k = 0; k < 2; ++k) {
        Plan& P = c.cycle[k];
        build(P, live, [&] {
          build_cycle(P, live, o);
          add_gather(P, live, gather_to);
        });
        c.ncycle = k + 1;
        if (level_state(live) == s0) break;
      }
      if (level_state(live) != s0) fail(INPAINT_E_DEVICE, "cycle plans do not return to their start state");
      upload({&c.cascade, &c.cycle[0], &c.cycle[1]}, &c.plan_dev, &c.plan_cap, s);
      HIPCHK(hipStreamSynchronize(s));
      if (!prof)
        for (int k = 0; k < c.ncycle; ++k) capture(c.cycle[k], c, prec, B);
    }
    HIPCHK(issue(c.cascade, prec, B, s, prof));
    std::vector<const Plan*> seq{&c.cascade};
    int cycles = 0;
    for (; cycles < nahead; ++cycles) {
      const Plan& P = c.cycle[cycles % c.ncycle];
      run_plan(P, prec, B, s);
      seq.push_back(&P);
    }
    if (ahead) {
      HIPCHK(issue(spec, prec, B, s, prof));
      HIPCHK(hipEventRecord(c.ev1, s));
    }
    HIPCHK(hipMemcpyAsync(c.flags_host, flags_src, (size_t)n * kFlagInts * sizeof(int),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ahead) {
      bool rejected = false;
      for (Member* m : all) {
        check_prepared(c.flags_host, m);
        rejected = rejected || m->status != INPAINT_OK;
      }
      if (rejected) {
        // an input check failed: solve again, waiting for the checks first
        for (Member* m : all) reset_member(m);
        c.expect = 0;
        return run_batch(all, o, tol, s, prof);
      }
    }
    bool done = apply_counted(c.flags_host, live, seq);
    // every channel stopped within the cycles run ahead: the device-selected
    // output has written every result
    written = ahead && done;
    // Float32 CG can stall above tol (its updates round away against |u|): the
    // CG schedules give up, not converged, once the largest relative residual
    // still iterating has not improved by 1 % in kCgStallTests tests.
    constexpr int kCgStallTests = 16;
    double best = INFINITY;
    int stalled = 0;
    while (!done && cycles < o.max_cycles) {
      const Plan& P = c.cycle[cycles % c.ncycle];
      if (prof)
        HIPCHK(issue(P, prec, B, s, prof));
      else
        run_plan(P, prec, B, s);
      seq.push_back(&P);
      ++cycles;
      HIPCHK(hipMemcpyAsync(c.flags_host, flags_src, (size_t)n * kFlagInts * sizeof(int),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      done = apply_counted(c.flags_host, live, seq);
      if (!done && cg_schedule(o.schedule)) {
        double worst = 0.0;
        for (Member* m : live)
          for (int ch = 0; ch < m->C; ++ch)
            if (m->final_cur[ch] < 0) worst = std::max(worst, m->rel[ch]);
        if (worst < 0.99 * best) {
          best = worst;
          stalled = 0;
        } else if (++stalled >= kCgStallTests) {
          break;
        }
      }
    }
    int need = 0;
    for (Member* m : live) need = std::max(need, m->cycles);
    c.expect = done ? need : 0;
    for (size_t i = 0; i < live.size(); ++i) finish_member(live[i], seq.back()->cur0[i]);
    if (!written) {
      Plan out;
      build_output(out, live);
      upload({&out}, &c.call_dev, &c.call_cap, s);
      HIPCHK(issue(out, prec, B, s, prof));
    }
  }
  if (!written) HIPCHK(hipEventRecord(c.ev1, s));
  for (Member* m : live)
    if (m->out_host)
      HIPCHK(hipMemcpyAsync(m->out, m->o_d, (size_t)m->W * m->H * m->C * sizeof(float),
                            hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, c.ev0, c.ev1));
  return ms;
}

}  // namespace inpaint

#define INPAINT_EXPORT __attribute__((visibility("default")))

extern "C" {

INPAINT_EXPORT int inpaint_solve_batched(const inpaint_problem* problems, int n, double tol,
                                         const inpaint_opts* opts, void* stream,
                                         inpaint_stats* stats) {
  return inpaint::guarded(
      [&] { return inpaint::solve_batched_impl(problems, n, tol, opts, stream, stats); });
}

}  // extern "C"
