// The single-problem solve without device allocation (inpaint_solve_noalloc):
// the same plans and kernels as inpaint_solve_ex, with the grid hierarchy and
// the launch arguments placed in one fixed device array per GPU instead of
// memory the library allocates, and no graph, stream, event or pinned buffer.
#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <mutex>

#include "batch.h"

namespace inpaint {
namespace {

constexpr size_t kScratchBytes = INPAINT_NOALLOC_SCRATCH_BYTES;
// Room kept after the plans for the output plan, which is built last (one
// OutputArgs and two offsets; checked when it is placed).
constexpr size_t kOutputReserve = 4096;

// The array.  In host code `scratch` names a host-side stand-in, not device
// memory: only the address hipGetSymbolAddress returns for the current device
// is ever passed to the device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DevScratch {
  std::mutex mu;           // one call at a time on this device
  unsigned char* ptr = nullptr;
};

std::mutex g_smu;
std::map<int, std::unique_ptr<DevScratch>> g_scratch;

// The device address of this device's array, looked up once per device with
// that device current.
DevScratch& device_scratch(int dev) {
  std::lock_guard<std::mutex> g(g_smu);
  auto& slot = g_scratch[dev];
  if (!slot) {
    auto d = std::make_unique<DevScratch>();
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(INPAINT_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    d->ptr = (unsigned char*)p;
    slot = std::move(d);
  }
  return *slot;
}

// Place the plans' argument arrays at dev + *off (256-byte aligned, bounded by
// limit) and copy them there.
void place(std::vector<Plan*> plans, unsigned char* dev, size_t* off, size_t limit, hipStream_t s) {
  size_t need = 0;
  for (Plan* p : plans) need += round_up(p->host.size(), 256);
  if (*off + need > limit)
    fail(INPAINT_E_INVALID, "the problem's grid hierarchy and launch arguments need " +
                                std::to_string(*off + need + kOutputReserve) +
                                " device bytes, more than the no-alloc array's " +
                                std::to_string(kScratchBytes));
  for (Plan* p : plans) {
    p->dev = dev + *off;
    if (!p->host.empty())
      HIPCHK(hipMemcpyAsync(p->dev, p->host.data(), p->host.size(), hipMemcpyHostToDevice, s));
    *off += round_up(p->host.size(), 256);
  }
}

void read_flags(int* host, const Workspace* ws, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(host, ws->relres, kFlagInts * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

int solve_noalloc_impl(const float* f, const uint8_t* mask, int W, int H, int C, double tol,
                       float* out, const inpaint_opts* opts, void* stream, inpaint_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  check_dims(f, mask, W, H, C);
  if (!out) fail(INPAINT_E_INVALID, "NULL pointer argument");
  if (!(tol > 0.0 && tol < 1.0)) fail(INPAINT_E_INVALID, "tol must lie in (0, 1)");
  Opts o = resolve(opts);
  o.profile = 0;
  if (cg_schedule(o.schedule))
    fail(INPAINT_E_INVALID, "inpaint_solve_noalloc runs the ORAS schedules only");
  check_geometry(W, H, o.B, o.o);
  const size_t nf = (size_t)W * H * C * sizeof(float);
  if (out != f && overlap(out, nf, f, nf)) fail(INPAINT_E_INVALID, "out partially overlaps f");
  if (overlap(out, nf, mask, (size_t)W * H)) fail(INPAINT_E_INVALID, "out overlaps mask");
  if (!is_device_ptr(f) || !is_device_ptr(mask) || !is_device_ptr(out))
    fail(INPAINT_E_INVALID, "inpaint_solve_noalloc takes device pointers only");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  DevScratch& ds = device_scratch(dev);
  std::lock_guard<std::mutex> lock(ds.mu);

  // the hierarchy at the start of the array (rejected here if it is too large)
  const Key k{dev, W, H, C, o.B, o.o, coarsest_side(o.B), o.prec};
  std::unique_ptr<Workspace> ws = bind_workspace(k, ds.ptr, kScratchBytes - kOutputReserve, s);
  Member m;
  m.W = W;
  m.H = H;
  m.C = C;
  m.ws = ws.get();
  m.R.reset(new Run{m.ws, o, s, C, tol});
  m.f_d = f;
  m.m_d = mask;
  m.o_d = out;
  m.out = out;
  m.final_cur.assign(C, -1);
  m.rel.assign(C, 0.0);
  const std::vector<Member*> ms{&m};

  // every plan is built on the host before any launch, so that a problem too
  // large for the array is rejected before device work starts
  Plan prep, cascade, cycle[2];
  build(prep, ms, [&] { build_prepare(prep, ms, o, nullptr); });
  build(cascade, ms, [&] { build_cascade(cascade, ms, o); });
  const std::vector<int> s0 = level_state(ms);
  int ncycle = 0;
  for (int c = 0; c < 2; ++c) {
    build(cycle[c], ms, [&] { build_cycle(cycle[c], ms, o); });
    ncycle = c + 1;
    if (level_state(ms) == s0) break;
  }
  if (level_state(ms) != s0) fail(INPAINT_E_DEVICE, "cycle plans do not return to their start state");
  size_t off = round_up(ws->bytes, 256);
  const size_t limit = kScratchBytes - kOutputReserve;
  place({&prep, &cascade, &cycle[0], &cycle[1]}, ds.ptr, &off, limit, s);

  int flags[kFlagInts];
  HIPCHK(issue(prep, o.prec, o.B, s));
  read_flags(flags, m.ws, s);
  check_prepared(flags, &m);
  if (m.status != INPAINT_OK) fail(m.status, m.msg);

  HIPCHK(issue(cascade, o.prec, o.B, s));
  std::vector<const Plan*> seq{&cascade};
  read_flags(flags, m.ws, s);
  bool done = apply_counted(flags, ms, seq);
  int cycles = 0;
  while (!done && cycles < o.max_cycles) {
    const Plan& P = cycle[cycles % ncycle];
    HIPCHK(issue(P, o.prec, o.B, s));
    seq.push_back(&P);
    ++cycles;
    read_flags(flags, m.ws, s);
    done = apply_counted(flags, ms, seq);
  }
  finish_member(&m, seq.back()->cur0[0]);
  Plan outp;
  build_output(outp, ms);
  place({&outp}, ds.ptr, &off, kScratchBytes, s);
  HIPCHK(issue(outp, o.prec, o.B, s));
  HIPCHK(hipStreamSynchronize(s));
  if (stats) {
    fill_stats(&m, *stats);
    stats->gpu_ms = (float)std::chrono::duration<double, std::milli>(
                        std::chrono::steady_clock::now() - t0)
                        .count();
  }
  g_err = m.status == INPAINT_OK ? "" : m.msg;
  return m.status;
}

}  // namespace
}  // namespace inpaint

#define INPAINT_EXPORT __attribute__((visibility("default")))

extern "C" {

INPAINT_EXPORT int inpaint_solve_noalloc(const float* f, const uint8_t* mask, int W, int H,
                                         int channels, double tol, float* out,
                                         const inpaint_opts* opts, void* stream,
                                         inpaint_stats* stats) {
  return inpaint::guarded([&] {
    return inpaint::solve_noalloc_impl(f, mask, W, H, channels, tol, out, opts, stream, stats);
  });
}

}  // extern "C"
