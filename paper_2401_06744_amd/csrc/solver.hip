// Host side of the inpainting library: workspaces (grid hierarchy in HBM),
// the cycle driver of Section 4.2 and the C ABI of include/inpaint.h.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>
#include <cstdlib>
#include <map>

#include "batch.h"
#include "driver.h"

namespace inpaint {

Opts resolve(const inpaint_opts* p) {
  Opts o;
  if (p) {
    if (p->struct_size != (int)sizeof(inpaint_opts))
      fail(INPAINT_E_INVALID, "inpaint_opts.struct_size must equal sizeof(inpaint_opts)");
    if (p->block) o.B = p->block;
    if (p->overlap) o.o = p->overlap;
    if (p->gamma != 0.0f) o.gamma = p->gamma;
    if (p->tau != 0.0f) o.tau = p->tau;
    if (p->max_local_iters) o.maxit = p->max_local_iters;
    o.schedule = p->schedule;
    if (p->max_cycles) o.max_cycles = p->max_cycles;
    if (p->pre_smooth) o.pre = p->pre_smooth < 0 ? 0 : p->pre_smooth;
    if (p->post_smooth) o.post = p->post_smooth < 0 ? 0 : p->post_smooth;
    o.rhs = p->rhs_restriction;
    if (p->coarse_tau != 0.0f) o.coarse_tau = p->coarse_tau;
    if (p->coarse_max_iters) o.coarse_maxit = p->coarse_max_iters;
    o.profile = p->profile;
    o.prec = p->precision;
  }
  if (o.prec != PREC_F32 && o.prec != PREC_F16 && o.prec != PREC_BF16)
    fail(INPAINT_E_INVALID, "unknown precision");
  if (o.B != 16 && o.B != 32 && o.B != 64) fail(INPAINT_E_INVALID, "block must be 16, 32 or 64");
  if (o.o < 2 || 2 * o.o > o.B) fail(INPAINT_E_INVALID, "overlap must satisfy 2 <= overlap <= block/2");
  // the overlap is twice the per-side halo of a block; with an even overlap
  // (and block) every block starts at an even column, which the grid passes'
  // pixel-pair accesses rely on
  if (o.o % 2 != 0) fail(INPAINT_E_INVALID, "overlap must be even (twice the per-side halo)");
  if (!(o.gamma > 0.0f && o.gamma <= 1.0f)) fail(INPAINT_E_INVALID, "gamma must lie in (0, 1]");
  if (!(o.tau >= 0.0f) || !std::isfinite(o.tau)) fail(INPAINT_E_INVALID, "tau must be finite and >= 0");
  if (o.maxit < 0 || o.coarse_maxit < 0) fail(INPAINT_E_INVALID, "iteration caps must be >= 0");
  if (o.schedule < INPAINT_SCHED_RFMG || o.schedule > INPAINT_SCHED_WARM)
    fail(INPAINT_E_INVALID, "unknown schedule");
  if (cg_schedule(o.schedule) && o.prec != PREC_F32)
    fail(INPAINT_E_INVALID, "the CG schedules run in float32 only");
  if (o.schedule == INPAINT_SCHED_CG_MULTILEVEL || o.schedule == INPAINT_SCHED_CG_MULTIGRID) {
    const int nu = o.schedule == INPAINT_SCHED_CG_MULTILEVEL ? kCgSmoothMultilevel : kCgSmoothMultigrid;
    if (!p || !p->pre_smooth) o.pre = nu;
    if (!p || !p->post_smooth) o.post = nu;
  }
  if (o.rhs != INPAINT_RHS_MODIFIED && o.rhs != INPAINT_RHS_NAIVE)
    fail(INPAINT_E_INVALID, "unknown rhs_restriction");
  if (o.pre > 16 || o.post > 16) fail(INPAINT_E_INVALID, "smoothing counts must be at most 16");
  if (!(o.coarse_tau >= 0.0f)) fail(INPAINT_E_INVALID, "coarse_tau must be >= 0");
  if (o.max_cycles < 0) fail(INPAINT_E_INVALID, "max_cycles must be >= 0");
  if (o.max_cycles == 0)
    o.max_cycles = (o.schedule == INPAINT_SCHED_RFMG || o.schedule == INPAINT_SCHED_FMG ||
                    o.schedule == INPAINT_SCHED_CG_MULTIGRID || o.schedule == INPAINT_SCHED_WARM)
                       ? 30
                   : cg_schedule(o.schedule) ? 500
                                             : 2000;
  return o;
}

Workspace::~Workspace() {
    int old = -1;
    (void)hipGetDevice(&old);
    (void)hipSetDevice(key.dev);
    if (base) (void)hipFree(base);
    if (stage_base) (void)hipFree(stage_base);
    if (cg_base) (void)hipFree(cg_base);
    if (host) (void)hipHostFree(host);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    if (old >= 0) (void)hipSetDevice(old);
  }

std::vector<std::pair<int, int>> level_sizes(int W, int H, int coarsest) {
  std::vector<std::pair<int, int>> s{{W, H}};
  while (s.back().first > coarsest || s.back().second > coarsest) {
    const auto [w, h] = s.back();
    s.push_back({(w + 1) / 2, (h + 1) / 2});
    if ((int)s.size() > kMaxLevels) break;
  }
  return s;
}

// Lay out the workspace of key k: the byte size of every buffer from offset 0
// (ws->bytes) and, when base is not null, the buffers' addresses in base.
static void lay_out(Workspace* ws, const Key& k, char* base) {
  const auto sizes = level_sizes(k.W, k.H, k.coarsest);
  if ((int)sizes.size() > kMaxLevels) fail(INPAINT_E_INVALID, "image too large for the level table");
  ws->key = k;
  ws->L = (int)sizes.size();
  const int C = k.C;
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t at = off;
    off = round_up(off + n, 256);
    return base ? base + at : nullptr;
  };
  size_t maxtiles = 1;
  for (int l = 0; l < ws->L; ++l) {
    Level& L = ws->lv[l];
    LevelView& v = L.v;
    v.W = sizes[l].first;
    v.H = sizes[l].second;
    v.P = (int)round_up((size_t)v.W, 64);
    v.plane = (size_t)v.H * v.P;
    v.B = k.B;
    v.o = k.o;
    v.nbx = num_blocks_axis(v.W, k.B, k.o);
    v.nby = num_blocks_axis(v.H, k.B, k.o);
    // the finest grid keeps float32 iterate, known values and residual; the
    // corrections and all coarser fields use the correction precision
    const size_t es = prec_bytes(k.prec);
    const size_t f = (size_t)C * v.plane * (l == 0 ? sizeof(float) : es);
    L.c = (uint8_t*)take(v.plane);
    L.b = (float*)take(f);
    L.u[0] = (float*)take(f);
    L.u[1] = (float*)take(f);
    // the precision form's finest grid keeps its residual in 16 bits (d, rh)
    // beside the correction e; the float32 residual is not needed there
    const bool corr = l == 0 && k.prec == PREC_F16 && ws->L > 1;
    L.r = corr ? nullptr : (float*)take(f);
    if (corr) {
      const size_t fe = (size_t)C * v.plane * es;
      L.e[0] = take(fe);
      L.e[1] = take(fe);
      L.d = take(fe);
      L.rh = take(fe);
    }
    L.contrib = (float*)take((size_t)C * v.nbx * v.nby * k.B * k.B * es);
    L.itot = (int*)take((size_t)2 * C * v.nbx * v.nby * sizeof(int));
    L.imax = L.itot ? L.itot + (size_t)C * v.nbx * v.nby : nullptr;
    // deferred norm partials: written by passes over this level or, for the
    // fused restriction, over the next finer one
    const size_t wt = std::max(pass_tiles(v), l > 0 ? pass_tiles(ws->lv[l - 1].v) : (size_t)0);
    L.dstride = wt <= Run::kDeferMax ? (int)wt : 0;
    L.dpart = L.dstride ? (double*)take((size_t)C * wt * sizeof(double)) : nullptr;
    maxtiles = std::max(maxtiles, pass_tiles(v));
  }
  ws->maxtiles = maxtiles;
  ws->partials = (double*)take((size_t)C * maxtiles * sizeof(double));
  ws->counters = (unsigned*)take((size_t)C * kCounterLines * 32 * sizeof(unsigned));
  ws->snorm = (double*)take((size_t)ws->L * C * sizeof(double));
  ws->den = (double*)take((size_t)C * sizeof(double));
  ws->rho = (float*)take((size_t)C * sizeof(float));
  // relres[4] doubles, active[4], status[4] and checks[4] ints: one block of
  // kFlagInts ints, so that a poll is a single copy
  char* flags = take(kFlagInts * sizeof(int));
  ws->relres = (double*)flags;
  ws->active = flags ? (int*)(flags + 32) : nullptr;
  ws->status = flags ? (int*)(flags + 48) : nullptr;
  ws->checks = flags ? (int*)(flags + 64) : nullptr;
  ws->cgstat = (unsigned long long*)take((size_t)kMaxLevels * C * 3 * sizeof(unsigned long long));
  ws->bytes = off;
}

void clear_workspace_state(Workspace* ws, hipStream_t s) {
  const int C = ws->key.C;
  // counters 0 (a whole number of doubles of zero bits), partials unset,
  // convergence-test counts 0
  static_assert((kCounterLines * 32 * sizeof(unsigned)) % sizeof(double) == 0, "counter block size");
  HIPCHK(launch_fill((double*)ws->counters, (size_t)C * kCounterLines * 32 * sizeof(unsigned) / sizeof(double),
                     0.0, s));
  HIPCHK(launch_fill(ws->partials, (size_t)C * ws->maxtiles, unset_partial(), s));
  HIPCHK(launch_fill((double*)ws->checks, 4 * sizeof(int) / sizeof(double), 0.0, s));
}

std::unique_ptr<Workspace> create_workspace(const Key& k, bool alloc) {
  check_geometry(k.W, k.H, k.B, k.o);
  auto ws = std::make_unique<Workspace>();
  lay_out(ws.get(), k, nullptr);
  if (!alloc) return ws;
  HIPCHK(hipMalloc(&ws->base, ws->bytes));
  lay_out(ws.get(), k, (char*)ws->base);
  clear_workspace_state(ws.get(), nullptr);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipHostMalloc(&ws->host, 4096, hipHostMallocDefault));
  HIPCHK(hipEventCreate(&ws->ev0));
  HIPCHK(hipEventCreate(&ws->ev1));
  return ws;
}

std::unique_ptr<Workspace> bind_workspace(const Key& k, void* base, size_t capacity, hipStream_t s) {
  check_geometry(k.W, k.H, k.B, k.o);
  auto ws = std::make_unique<Workspace>();
  lay_out(ws.get(), k, nullptr);
  if (ws->bytes > capacity)
    fail(INPAINT_E_INVALID, "the problem's grid hierarchy needs " + std::to_string(ws->bytes) +
                                " device bytes, more than the " + std::to_string(capacity) + " available");
  lay_out(ws.get(), k, (char*)base);
  clear_workspace_state(ws.get(), s);
  return ws;
}

size_t workspace_bytes(const Key& k) { return create_workspace(k, false)->bytes; }

namespace {

// Workspaces of single and batched solves, cached between calls per key and
// bounded in total device bytes: an idle workspace is freed, least recently
// used first, when a new one (or a lease's end) would leave the cache above
// the limit.  A workspace in use is never freed.
std::mutex g_mu;
std::map<Key, std::vector<std::unique_ptr<Workspace>>> g_cache;
unsigned long long g_serial = 0, g_tick = 0;
size_t g_limit = 0;  // 0 until first use: then INPAINT_CACHE_LIMIT_MB or the default

constexpr size_t kDefaultCacheLimit = (size_t)16 << 30;

size_t cache_limit_locked() {
  if (g_limit == 0) {
    g_limit = kDefaultCacheLimit;
    if (const char* e = std::getenv("INPAINT_CACHE_LIMIT_MB")) {
      const long long mb = std::atoll(e);
      if (mb > 0) g_limit = (size_t)mb << 20;
    }
  }
  return g_limit;
}

size_t footprint(const Workspace& w) {
  size_t b = w.bytes;
  if (w.stage_base) b += w.stage_bytes;
  if (w.cg_base) b += w.cg_bytes;
  return b;
}

size_t cached_bytes_locked() {
  size_t t = 0;
  for (auto& kv : g_cache)
    for (auto& w : kv.second) t += footprint(*w);
  return t;
}

// Free idle workspaces, least recently used first, until `need` more bytes
// fit under the limit (or nothing idle is left).
void trim_locked(size_t need) {
  const size_t limit = cache_limit_locked();
  size_t total = cached_bytes_locked();
  while (total + need > limit) {
    Workspace* lru = nullptr;
    for (auto& kv : g_cache)
      for (auto& w : kv.second)
        if (!w->busy && (!lru || w->last_use < lru->last_use)) lru = w.get();
    if (!lru) return;
    total -= footprint(*lru);
    auto& vec = g_cache[lru->key];
    for (auto it = vec.begin(); it != vec.end(); ++it)
      if (it->get() == lru) {
        vec.erase(it);  // frees the device memory (every call has synchronised its stream)
        break;
      }
    if (vec.empty()) g_cache.erase(lru->key);
  }
}

}  // namespace

Lease::~Lease() {
  if (ws) {
    std::lock_guard<std::mutex> g(g_mu);
    ws->busy = false;
    trim_locked(0);
  }
}

void acquire(Lease& lease, int W, int H, int C, int B, int o, int coarsest, int prec) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const Key k{dev, W, H, C, B, o, coarsest, prec};
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_cache.find(k);
    if (it != g_cache.end())
      for (auto& w : it->second)
        if (!w->busy) {
          w->busy = true;
          w->last_use = ++g_tick;
          lease.ws = w.get();
          return;
        }
    trim_locked(workspace_bytes(k));
  }
  auto ws = create_workspace(k);
  std::lock_guard<std::mutex> g(g_mu);
  ws->busy = true;
  ws->serial = ++g_serial;
  ws->last_use = ++g_tick;
  lease.ws = ws.get();
  g_cache[k].push_back(std::move(ws));
}

size_t set_cache_limit(size_t limit) {
  std::lock_guard<std::mutex> g(g_mu);
  if (limit) g_limit = limit;
  trim_locked(0);
  return cached_bytes_locked();
}

void ensure_staging(Workspace* ws) {
  if (ws->stage_base) return;
  const size_t n = (size_t)ws->key.W * ws->key.H;
  const size_t fb = round_up(n * ws->key.C * sizeof(float), 256);
  HIPCHK(hipMalloc(&ws->stage_base, 2 * fb + round_up(n, 256)));
  ws->stage_bytes = 2 * fb + round_up(n, 256);
  ws->f_dev = (float*)ws->stage_base;
  ws->o_dev = (float*)((char*)ws->stage_base + fb);
  ws->m_dev = (uint8_t*)((char*)ws->stage_base + 2 * fb);
}

void ensure_cg(Workspace* ws) {
  if (ws->cg_base) return;
  const Level& L0 = ws->lv[0];
  const size_t fb = round_up((size_t)ws->key.C * L0.v.plane * sizeof(float), 256);
  HIPCHK(hipMalloc(&ws->cg_base, 3 * fb + 256));
  ws->cg_bytes = 3 * fb + 256;
  char* b = (char*)ws->cg_base;
  ws->cg_p[0] = (float*)b;
  ws->cg_p[1] = (float*)(b + fb);
  ws->cg_q = (float*)(b + 2 * fb);
  ws->cgs = (double*)(b + 3 * fb);
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

namespace {

__global__ void k_reset(int* active, int* status, unsigned long long* cgstat, int C) {
  const int t = threadIdx.x;
  if (t < C) active[t] = 1;
  if (t < 4) status[t] = 0;
  if (t < kKnownWords) status[kKnownAt + t] = 0;
  for (int i = t; i < 3 * C * kMaxLevels; i += blockDim.x) cgstat[i] = 0;
}

}  // namespace

// Stage (f, mask) into level 0 and build the hierarchy.  Returns after the
// input checks have been read back.
void prepare(Run& R, const float* f_d, const uint8_t* m_d, bool hierarchy, bool write_u) {
  Workspace* ws = R.ws;
  const int C = R.C;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, R.s, ws->active, ws->status, ws->cgstat, C);
  HIPCHK(hipGetLastError());
  if (R.o.profile)
    for (int l = 0; l < ws->L; ++l) {
      const Level& L = ws->lv[l];
      // two int arrays of C*nblk entries = C*nblk doubles of zero bits
      HIPCHK(launch_fill((double*)L.itot, (size_t)C * L.v.nbx * L.v.nby, 0.0, R.s));
    }
  Level& L0 = ws->lv[0];
  L0.cur = 0;
  // staging, input checks and the reference residual ||b - A C f|| (denominator
  // of the relative residual)
  NormOut den = R.norm(0, false);
  den.mode = NORM_FULL;
  den.out = ws->den;
  den.rho = ws->rho;
  den.inv_n = 1.0 / ((double)ws->key.W * (double)ws->key.H);
  R.timed(INPAINT_K_STAGE, 0, [&] {
    return launch_stage(f_d, m_d, ws->key.W, ws->key.H, C, ws->key.W, L0.v, L0.c, L0.b,
                        (write_u || ws->L == 1) ? L0.u[0] : nullptr, ws->status, den, R.s);
  });
  if (hierarchy) {
    for (int l = 0; l + 1 < ws->L; ++l) {
      Level& F = ws->lv[l];
      Level& Cl = ws->lv[l + 1];
      Cl.cur = 0;
      R.timed(INPAINT_K_PYRAMID, l, [&] {
        return launch_rhs_down(F.v, F.c, F.b, Cl.v, Cl.c, Cl.b, C,
                               R.o.rhs == INPAINT_RHS_NAIVE ? 1 : 0, R.prec(), l == 0 ? 1 : 0, R.s);
      });
    }
  }
  int* h = (int*)ws->host;
  HIPCHK(hipMemcpyAsync(h, ws->status, (kKnownAt + kKnownWords) * sizeof(int), hipMemcpyDeviceToHost, R.s));
  HIPCHK(hipStreamSynchronize(R.s));
  const int st = input_checks(h);
  if (st & 1) fail(INPAINT_E_INVALID, "f is not finite at a known pixel");
  if (!(st & 2)) fail(INPAINT_E_EMPTY_MASK, "mask has no known pixel: the system is singular");
}

void check_dims(const void* a, const void* b, int W, int H, int C) {
  if (!a || !b) fail(INPAINT_E_INVALID, "NULL pointer argument");
  if (W < 1 || H < 1) fail(INPAINT_E_INVALID, "W and H must be >= 1");
  if (C < 1 || C > kMaxChannels) fail(INPAINT_E_INVALID, "channels must lie in [1, 4]");
  if ((long long)W * H > (1LL << 31)) fail(INPAINT_E_INVALID, "image too large");
}

void check_geometry(int W, int H, int B, int o) {
  // Offsets inside one channel's fields and inside one channel's weighted
  // block corrections are 32-bit in the kernels, and a pixel index is split
  // into blocks through a float reciprocal that is exact below 2^24.
  if (std::max(W, H) >= (1 << 24)) fail(INPAINT_E_INVALID, "image sides must be below 2^24 pixels");
  const long long P = (long long)round_up((size_t)W, 64);
  if ((long long)H * P > (long long)INT32_MAX)
    fail(INPAINT_E_INVALID, "image too large: a channel's padded plane exceeds 32-bit offsets");
  const long long nb = (long long)num_blocks_axis(W, B, o) * num_blocks_axis(H, B, o) * B * B;
  if (nb > (long long)INT32_MAX)
    fail(INPAINT_E_INVALID, "image too large: a channel's block corrections exceed 32-bit offsets");
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

int solve_impl(const float* f, const uint8_t* mask, int W, int H, int C, double tol, float* out,
               const inpaint_opts* opts, void* stream, inpaint_stats* stats) {
  check_dims(f, mask, W, H, C);
  if (!out) fail(INPAINT_E_INVALID, "NULL pointer argument");
  if (!(tol > 0.0 && tol < 1.0)) fail(INPAINT_E_INVALID, "tol must lie in (0, 1)");
  const Opts o = resolve(opts);
  check_geometry(W, H, o.B, o.o);
  const size_t nf = (size_t)W * H * C * sizeof(float);
  if (out != f && overlap(out, nf, f, nf)) fail(INPAINT_E_INVALID, "out partially overlaps f");
  if (overlap(out, nf, mask, (size_t)W * H)) fail(INPAINT_E_INVALID, "out overlaps mask");
  hipStream_t s = (hipStream_t)stream;
  Member m;
  acquire(m.lease, W, H, C, o.B, o.o, coarsest_side(o.B), o.prec);
  const inpaint_problem p{f, mask, W, H, C, out};
  init_member(m, p, m.lease.ws, o, tol, s);
  Workspace* ws = m.ws;
  Prof prof;
  prof.pool = &ws->evpool;
  if (o.profile)
    for (int l = 0; l < ws->L; ++l) {
      const Level& L = ws->lv[l];
      // two int arrays of C*nblk entries = C*nblk doubles of zero bits
      HIPCHK(launch_fill((double*)L.itot, (size_t)C * L.v.nbx * L.v.nby, 0.0, s));
    }
  const float ms = run_batch({&m}, o, tol, s, o.profile ? &prof : nullptr);
  if (m.status == INPAINT_E_INVALID || m.status == INPAINT_E_EMPTY_MASK) fail(m.status, m.msg);
  if (stats) {
    fill_stats(&m, *stats);
    stats->gpu_ms = ms;
    if (o.profile) {
      for (int l = 0; l < ws->L; ++l)
        HIPCHK(launch_cg_stats(ws->lv[l].v, ws->lv[l].itot, ws->lv[l].imax, C,
                               ws->cgstat + (size_t)l * C * 3, s));
      std::vector<unsigned long long> cg((size_t)3 * C * ws->L, 0);
      HIPCHK(hipMemcpyAsync(cg.data(), ws->cgstat, cg.size() * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      unsigned long long tot = 0, mx = 0, fin = 0, finpx = 0;
      for (int l = 0; l < ws->L; ++l)
        for (int ch = 0; ch < C; ++ch) {
          const unsigned long long* c3 = &cg[((size_t)l * C + ch) * 3];
          tot += c3[0];
          mx = std::max(mx, c3[1]);
          if (l == 0) {
            fin += c3[0];
            finpx += c3[2];
          }
        }
      stats->local_cg_mean = m.blocks ? (double)tot / (double)m.blocks : 0.0;
      stats->local_cg_max = (int)mx;
      stats->local_cg_finest = (double)fin;
      stats->finest_cg_pixel_iters = (double)finpx;
      for (const auto& rc : prof.recs) {
        float kms = 0.0f;
        HIPCHK(hipEventElapsedTime(&kms, rc.a, rc.b));
        stats->kernel_ms[rc.cls] += kms;
        stats->kernel_calls[rc.cls] += 1;
      }
    }
  }
  g_err = m.status == INPAINT_OK ? "" : m.msg;
  return m.status;
}

// Copy a host [C][H][W] array into a pitched level field.
void upload_field(const float* src, const Level& L, float* dst, int C, hipStream_t s) {
  for (int ch = 0; ch < C; ++ch)
    HIPCHK(hipMemcpy2DAsync(dst + (size_t)ch * L.v.plane, (size_t)L.v.P * sizeof(float),
                            src + (size_t)ch * L.v.W * L.v.H, (size_t)L.v.W * sizeof(float),
                            (size_t)L.v.W * sizeof(float), L.v.H, hipMemcpyHostToDevice, s));
}
void download_field(const float* src, const Level& L, float* dst, int C, hipStream_t s) {
  for (int ch = 0; ch < C; ++ch)
    HIPCHK(hipMemcpy2DAsync(dst + (size_t)ch * L.v.W * L.v.H, (size_t)L.v.W * sizeof(float),
                            src + (size_t)ch * L.v.plane, (size_t)L.v.P * sizeof(float),
                            (size_t)L.v.W * sizeof(float), L.v.H, hipMemcpyDeviceToHost, s));
}

}  // namespace inpaint

using namespace inpaint;

#define INPAINT_EXPORT __attribute__((visibility("default")))

extern "C" {

INPAINT_EXPORT int inpaint_solve(const float* f, const uint8_t* mask, int W, int H, int channels, double tol,
                  float* out) {
  return guarded([&] { return solve_impl(f, mask, W, H, channels, tol, out, nullptr, nullptr, nullptr); });
}

INPAINT_EXPORT int inpaint_solve_ex(const float* f, const uint8_t* mask, int W, int H, int channels, double tol,
                     float* out, const inpaint_opts* opts, void* stream, inpaint_stats* stats) {
  return guarded([&] { return solve_impl(f, mask, W, H, channels, tol, out, opts, stream, stats); });
}

INPAINT_EXPORT int inpaint_cache_limit(size_t limit_bytes, size_t* cached_bytes) {
  return guarded([&] {
    const size_t b = set_cache_limit(limit_bytes);
    if (cached_bytes) *cached_bytes = b;
    return INPAINT_OK;
  });
}

INPAINT_EXPORT const char* inpaint_last_error(void) { return g_err.c_str(); }

INPAINT_EXPORT const char* inpaint_version(void) { return "inpaint-mi355x 0.1 (gfx950)"; }

INPAINT_EXPORT int inpaint_rel_res(const float* u, const float* f, const uint8_t* mask, int W, int H, int channels,
                    double* rel_res_out) {
  return guarded([&] {
    check_dims(f, mask, W, H, channels);
    if (!u || !rel_res_out) fail(INPAINT_E_INVALID, "NULL pointer argument");
    Lease lease;
    acquire(lease, W, H, channels, 32, 6, 1 << 30);
    Workspace* ws = lease.ws;
    ensure_staging(ws);
    hipStream_t s = nullptr;
    const size_t nf = (size_t)W * H * channels * sizeof(float);
    const float* f_d = f;
    const uint8_t* m_d = mask;
    if (!is_device_ptr(f)) {
      HIPCHK(hipMemcpyAsync(ws->f_dev, f, nf, hipMemcpyHostToDevice, s));
      f_d = ws->f_dev;
    }
    if (!is_device_ptr(mask)) {
      HIPCHK(hipMemcpyAsync(ws->m_dev, mask, (size_t)W * H, hipMemcpyHostToDevice, s));
      m_d = ws->m_dev;
    }
    Opts o;
    Run R{ws, o, s, channels, 0.5};
    prepare(R, f_d, m_d, false, false);
    Level& L0 = ws->lv[0];
    const hipMemcpyKind kind = is_device_ptr(u) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int ch = 0; ch < channels; ++ch)
      HIPCHK(hipMemcpy2DAsync(L0.u[1] + (size_t)ch * L0.v.plane, (size_t)L0.v.P * sizeof(float),
                              u + (size_t)ch * W * H, (size_t)W * sizeof(float),
                              (size_t)W * sizeof(float), H, kind, s));
    L0.cur = 1;
    R.residual(0, true);  // the full in-pass reduction writes the norm read below
    std::vector<double> sn(channels), den(channels);
    HIPCHK(hipMemcpyAsync(sn.data(), ws->snorm, channels * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(den.data(), ws->den, channels * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int ch = 0; ch < channels; ++ch)
      rel_res_out[ch] = den[ch] > 0 ? std::sqrt(sn[ch] / den[ch]) : (sn[ch] > 0 ? INFINITY : 0.0);
    return INPAINT_OK;
  });
}

INPAINT_EXPORT int inpaint_hierarchy_size(int W, int H, int block, int* levels_out, size_t* pixels_out) {
  return guarded([&] {
    if (W < 1 || H < 1 || block < 1) fail(INPAINT_E_INVALID, "W, H and block must be >= 1");
    const auto sz = level_sizes(W, H, block);
    if ((int)sz.size() > kMaxLevels) fail(INPAINT_E_INVALID, "image too large for the level table");
    size_t n = 0;
    for (auto& p : sz) n += (size_t)p.first * p.second;
    if (levels_out) *levels_out = (int)sz.size();
    if (pixels_out) *pixels_out = n;
    return INPAINT_OK;
  });
}

INPAINT_EXPORT int inpaint_debug_pyramid(const float* f, const uint8_t* mask, int W, int H, int channels, int block,
                          int rhs_restriction, int* levels_out, int* sizes_out, uint8_t* masks_out,
                          float* rhs_out) {
  return guarded([&] {
    check_dims(f, mask, W, H, channels);
    if (block < 1) fail(INPAINT_E_INVALID, "block must be >= 1");
    if (rhs_restriction != INPAINT_RHS_MODIFIED && rhs_restriction != INPAINT_RHS_NAIVE)
      fail(INPAINT_E_INVALID, "unknown rhs_restriction");
    Lease lease;
    acquire(lease, W, H, channels, 32, 6, block);
    Workspace* ws = lease.ws;
    ensure_staging(ws);
    hipStream_t s = nullptr;
    HIPCHK(hipMemcpyAsync(ws->f_dev, f, (size_t)W * H * channels * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws->m_dev, mask, (size_t)W * H, hipMemcpyHostToDevice, s));
    Opts o;
    o.rhs = rhs_restriction;
    Run R{ws, o, s, channels, 0.5};
    prepare(R, ws->f_dev, ws->m_dev, true, false);
    if (levels_out) *levels_out = ws->L;
    size_t mo = 0, ro = 0;
    for (int l = 0; l < ws->L; ++l) {
      const Level& L = ws->lv[l];
      if (sizes_out) {
        sizes_out[2 * l] = L.v.W;
        sizes_out[2 * l + 1] = L.v.H;
      }
      if (masks_out)
        HIPCHK(hipMemcpy2DAsync(masks_out + mo, L.v.W, L.c, L.v.P, L.v.W, L.v.H, hipMemcpyDeviceToHost, s));
      if (rhs_out) download_field(L.b, L, rhs_out + ro, channels, s);
      mo += (size_t)L.v.W * L.v.H;
      ro += (size_t)L.v.W * L.v.H * channels;
    }
    HIPCHK(hipStreamSynchronize(s));
    return INPAINT_OK;
  });
}

INPAINT_EXPORT int inpaint_debug_oras_step(const float* u_in, const float* f, const uint8_t* mask, int W, int H,
                            int channels, const inpaint_opts* opts, float* u_out) {
  return guarded([&] {
    check_dims(f, mask, W, H, channels);
    if (!u_in || !u_out) fail(INPAINT_E_INVALID, "NULL pointer argument");
    const Opts o = resolve(opts);
    Lease lease;
    acquire(lease, W, H, channels, o.B, o.o, 1 << 30);
    Workspace* ws = lease.ws;
    ensure_staging(ws);
    hipStream_t s = nullptr;
    HIPCHK(hipMemcpyAsync(ws->f_dev, f, (size_t)W * H * channels * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws->m_dev, mask, (size_t)W * H, hipMemcpyHostToDevice, s));
    Run R{ws, o, s, channels, 0.5};
    prepare(R, ws->f_dev, ws->m_dev, false, false);
    Level& L0 = ws->lv[0];
    upload_field(u_in, L0, L0.u[0], channels, s);
    L0.cur = 0;
    R.residual(0, false);
    R.oras(0, false);
    download_field(L0.u[L0.cur], L0, u_out, channels, s);
    HIPCHK(hipStreamSynchronize(s));
    return INPAINT_OK;
  });
}

INPAINT_EXPORT int inpaint_debug_restrict(const float* r_f, const uint8_t* mask_c, int Wf, int Hf, float* r_c) {
  return guarded([&] {
    if (!r_f || !mask_c || !r_c) fail(INPAINT_E_INVALID, "NULL pointer argument");
    if (Wf < 2 && Hf < 2) fail(INPAINT_E_INVALID, "the fine grid must have more than one pixel");
    check_dims(r_f, mask_c, Wf, Hf, 1);
    Lease lease;
    acquire(lease, Wf, Hf, 1, 32, 6, 1);
    Workspace* ws = lease.ws;
    hipStream_t s = nullptr;
    Level& F = ws->lv[0];
    Level& Cl = ws->lv[1];
    upload_field(r_f, F, F.r, 1, s);
    HIPCHK(hipMemcpy2DAsync(Cl.c, Cl.v.P, mask_c, Cl.v.W, Cl.v.W, Cl.v.H, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, ws->active, ws->status, ws->cgstat, 1);
    HIPCHK(hipGetLastError());
    Opts o;
    Run R{ws, o, s, 1, 0.5};
    Cl.cur = 0;
    R.restrict_to(0);
    download_field(Cl.b, Cl, r_c, 1, s);
    HIPCHK(hipStreamSynchronize(s));
    return INPAINT_OK;
  });
}

INPAINT_EXPORT int inpaint_debug_prolong(const float* u_c, int Wf, int Hf, const uint8_t* mask_f, const float* b_f,
                          const float* u_in, int mode, float* u_out) {
  return guarded([&] {
    if (!u_c || !mask_f || !b_f || !u_out || (mode == 1 && !u_in))
      fail(INPAINT_E_INVALID, "NULL pointer argument");
    if (mode != 0 && mode != 1) fail(INPAINT_E_INVALID, "mode must be 0 or 1");
    if (Wf < 2 && Hf < 2) fail(INPAINT_E_INVALID, "the fine grid must have more than one pixel");
    check_dims(u_c, mask_f, Wf, Hf, 1);
    Lease lease;
    acquire(lease, Wf, Hf, 1, 32, 6, 1);
    Workspace* ws = lease.ws;
    hipStream_t s = nullptr;
    Level& F = ws->lv[0];
    Level& Cl = ws->lv[1];
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, ws->active, ws->status, ws->cgstat, 1);
    HIPCHK(hipGetLastError());
    upload_field(u_c, Cl, Cl.u[0], 1, s);
    Cl.cur = 0;
    HIPCHK(hipMemcpy2DAsync(F.c, F.v.P, mask_f, F.v.W, F.v.W, F.v.H, hipMemcpyHostToDevice, s));
    upload_field(b_f, F, F.b, 1, s);
    upload_field(mode == 1 ? u_in : b_f, F, F.u[0], 1, s);
    F.cur = 0;
    Opts o;
    Run R{ws, o, s, 1, 0.5};
    R.prolong(0, mode == 0 ? PASS_PSOL : PASS_PCORR, false);
    download_field(F.u[F.cur], F, u_out, 1, s);
    HIPCHK(hipStreamSynchronize(s));
    return INPAINT_OK;
  });
}

}  // extern "C"
