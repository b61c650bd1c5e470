// Autotuner of the batched solve: picks the block side, overlap, Robin weight,
// local CG tolerance and cycle schedule for a set of problems by timing
// batched solves of those problems (coordinate descent from the caller's
// options).  Choices are cached per workload signature in memory and, when
// INPAINT_AUTOTUNE_CACHE names a file, in that file (one line per signature).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <tuple>

#include "batch.h"

namespace inpaint {

int solve_batched_impl(const inpaint_problem* probs, int n, double tol, const inpaint_opts* opts,
                       void* stream, inpaint_stats* stats);

namespace {

struct Choice {
  int block, overlap, schedule;
  float gamma, tau;
  double ms;
};

std::mutex g_tmu;
std::map<std::string, Choice> g_tcache;
bool g_tloaded = false;

// Fraction of known pixels of a mask in host or device memory.
double mask_density(const uint8_t* m, int W, int H, hipStream_t s) {
  const size_t n = (size_t)W * H;
  std::vector<uint8_t> h;
  const uint8_t* p = m;
  if (is_device_ptr(m)) {
    h.resize(n);
    HIPCHK(hipMemcpyAsync(h.data(), m, n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    p = h.data();
  }
  size_t k = 0;
  for (size_t i = 0; i < n; ++i) k += p[i] != 0;
  return (double)k / (double)n;
}

// Workload signature: the device, every resolved option, the tolerance, and
// per problem its shape and mask density (in half-octave buckets: the local
// problems' difficulty follows the size of the unknown regions).
std::string signature(const inpaint_problem* p, int n, double tol, const Opts& o, int dev,
                      hipStream_t s) {
  std::vector<std::tuple<int, int, int, int>> shapes;
  for (int i = 0; i < n; ++i) {
    const double d = mask_density(p[i].mask, p[i].W, p[i].H, s);
    const int bucket = d > 0.0 ? (int)std::floor(2.0 * std::log2(d)) : -1000;
    shapes.emplace_back(p[i].W, p[i].H, p[i].channels, bucket);
  }
  std::sort(shapes.begin(), shapes.end());
  std::ostringstream k;
  char t[160];
  std::snprintf(t, sizeof t,
                "dev=%d;prec=%d;tol=%.17g;B=%d;o=%d;gamma=%.9g;tau=%.9g;maxit=%d;sched=%d;cycles=%d;"
                "pre=%d;post=%d;rhs=%d;ctau=%.9g;cmaxit=%d;n=%d",
                dev, o.prec, tol, o.B, o.o, (double)o.gamma, (double)o.tau, o.maxit, o.schedule,
                o.max_cycles, o.pre, o.post, o.rhs, (double)o.coarse_tau, o.coarse_maxit, n);
  k << t;
  for (auto& v : shapes)
    k << ";" << std::get<0>(v) << "x" << std::get<1>(v) << "x" << std::get<2>(v) << "d" << std::get<3>(v);
  return k.str();
}

const char* cache_file() {
  const char* f = std::getenv("INPAINT_AUTOTUNE_CACHE");
  return (f && *f) ? f : nullptr;
}

inpaint_opts to_opts(const inpaint_opts& base, const Choice& c);

bool valid(const Choice& c) {
  inpaint_opts o{};
  o.struct_size = sizeof(inpaint_opts);
  const inpaint_opts t = to_opts(o, c);
  const std::string keep = g_err;
  try {
    (void)resolve(&t);
  } catch (const Fail&) {
    g_err = keep;
    return false;
  }
  return (c.schedule == INPAINT_SCHED_RFMG || c.schedule == INPAINT_SCHED_FMG) && c.ms > 0.0;
}

void load_file() {
  if (g_tloaded) return;
  g_tloaded = true;
  const char* fn = cache_file();
  if (!fn) return;
  std::ifstream in(fn);
  std::string line;
  while (std::getline(in, line)) {
    const size_t tab = line.find('\t');
    if (tab == std::string::npos) continue;
    Choice c{};
    std::istringstream v(line.substr(tab + 1));
    if (!(v >> c.block >> c.overlap >> c.gamma >> c.tau >> c.schedule >> c.ms)) continue;
    // an entry the current library would reject (a stale or edited file) is skipped
    if (!valid(c)) continue;
    g_tcache[line.substr(0, tab)] = c;
  }
}

void save_file(const std::string& key, const Choice& c) {
  const char* fn = cache_file();
  if (!fn) return;
  std::ofstream out(fn, std::ios::app);
  out << key << '\t' << c.block << ' ' << c.overlap << ' ' << c.gamma << ' ' << c.tau << ' '
      << c.schedule << ' ' << c.ms << '\n';
}

inpaint_opts to_opts(const inpaint_opts& base, const Choice& c) {
  inpaint_opts o = base;
  o.struct_size = sizeof(inpaint_opts);
  o.block = c.block;
  o.overlap = c.overlap;
  o.gamma = c.gamma;
  o.tau = c.tau;
  o.schedule = c.schedule;
  return o;
}

}  // namespace

int autotune_impl(const inpaint_problem* probs, int n, double tol, const inpaint_opts* base_p,
                  void* stream, inpaint_opts* best, double* best_ms) {
  if (!best) fail(INPAINT_E_INVALID, "NULL output options");
  const Opts ob = resolve(base_p);  // validates
  inpaint_opts base{};
  if (base_p) base = *base_p;
  base.struct_size = sizeof(inpaint_opts);
  if (!probs || n < 1) fail(INPAINT_E_INVALID, "no problems to tune on");
  for (int i = 0; i < n; ++i) validate_problem(probs[i], i, ob);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const std::string key = signature(probs, n, tol, ob, dev, (hipStream_t)stream);
  {
    std::lock_guard<std::mutex> g(g_tmu);
    load_file();
    auto it = g_tcache.find(key);
    if (it != g_tcache.end()) {
      *best = to_opts(base, it->second);
      if (best_ms) *best_ms = it->second.ms;
      return INPAINT_OK;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  // wall time of one batched solve: median of three after a warm-up run; a
  // candidate that leaves any problem unconverged is out
  auto measure = [&](const Choice& c) -> double {
    const inpaint_opts o = to_opts(base, c);
    if (solve_batched_impl(probs, n, tol, &o, stream, nullptr) != INPAINT_OK) return INFINITY;
    double t[3];
    for (double& v : t) {
      const auto a = std::chrono::steady_clock::now();
      if (solve_batched_impl(probs, n, tol, &o, stream, nullptr) != INPAINT_OK) return INFINITY;
      HIPCHK(hipStreamSynchronize(s));
      v = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
    }
    std::sort(t, t + 3);
    return t[1];
  };
  Choice cur{ob.B, ob.o, ob.schedule, ob.gamma, ob.tau, 0.0};
  if (cur.schedule != INPAINT_SCHED_RFMG && cur.schedule != INPAINT_SCHED_FMG) cur.schedule = INPAINT_SCHED_RFMG;
  cur.ms = measure(cur);
  auto try_values = [&](auto setter, const auto& values) {
    for (const auto& v : values) {
      Choice c = cur;
      setter(c, v);
      if (c.overlap < 2 || 2 * c.overlap > c.block) continue;
      if (c.block == cur.block && c.overlap == cur.overlap && c.schedule == cur.schedule &&
          c.gamma == cur.gamma && c.tau == cur.tau)
        continue;
      c.ms = measure(c);
      if (c.ms < cur.ms) cur = c;
    }
  };
  const int schedules[] = {INPAINT_SCHED_RFMG, INPAINT_SCHED_FMG};
  const int blocks[] = {16, 32, 64};
  const int overlaps[] = {2, 4, 6, 8};
  const float gammas[] = {0.3f, 0.5f, 0.7f};
  const float taus[] = {0.002f, 0.005f, 0.01f};
  try_values([](Choice& c, int v) { c.schedule = v; }, schedules);
  try_values([](Choice& c, int v) {
    c.block = v;
    if (2 * c.overlap > v) c.overlap = v / 4;
  }, blocks);
  try_values([](Choice& c, int v) { c.overlap = v; }, overlaps);
  try_values([](Choice& c, float v) { c.gamma = v; }, gammas);
  try_values([](Choice& c, float v) { c.tau = v; }, taus);
  if (!std::isfinite(cur.ms)) fail(INPAINT_E_DIVERGED, "no candidate converged on every problem");
  {
    std::lock_guard<std::mutex> g(g_tmu);
    g_tcache[key] = cur;
    save_file(key, cur);
  }
  *best = to_opts(base, cur);
  if (best_ms) *best_ms = cur.ms;
  return INPAINT_OK;
}

}  // namespace inpaint

#define INPAINT_EXPORT __attribute__((visibility("default")))

extern "C" {

INPAINT_EXPORT int inpaint_autotune(const inpaint_problem* problems, int n, double tol,
                                    const inpaint_opts* base, void* stream, inpaint_opts* best,
                                    double* best_ms) {
  return inpaint::guarded(
      [&] { return inpaint::autotune_impl(problems, n, tol, base, stream, best, best_ms); });
}

}  // extern "C"
