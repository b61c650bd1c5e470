// Host-side driver shared by the single-problem, batched and serving entry
// points: options, workspaces (the grid hierarchy of one problem in HBM), the
// cycle driver's argument builders and the input staging.  Internal; the
// public ABI is include/inpaint.h.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "errors.h"
#include "inpaint.h"
#include "kernels.h"

namespace inpaint {


#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      fail(e_ == hipErrorOutOfMemory ? INPAINT_E_NOMEM : INPAINT_E_DEVICE,        \
           std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline int num_blocks_axis(int n, int B, int o) { return n <= B ? 1 : (n - o + (B - o) - 1) / (B - o); }

// Side of the coarsest grid of a hierarchy with ORAS block side B: the level
// rule halves until both sides are at most B (Section 4.4), except that a
// coarsest grid is at most 32 x 32, which one wavefront solves.
inline int coarsest_side(int B) { return B < 32 ? B : 32; }

// ---------------------------------------------------------------------------
// options
// ---------------------------------------------------------------------------

struct Opts {
  int B = 32, o = 6;
  float gamma = 0.5f, tau = 0.005f;
  int maxit = 16;
  int schedule = INPAINT_SCHED_RFMG;
  int max_cycles = 0;
  int pre = 1, post = 1;
  int rhs = INPAINT_RHS_MODIFIED;
  float coarse_tau = 1e-8f;
  int coarse_maxit = 256;
  int profile = 0;
  int prec = PREC_F32;
};

// The comparison schedules built on conjugate gradients.
inline bool cg_schedule(int s) {
  return s == INPAINT_SCHED_CG || s == INPAINT_SCHED_CG_MULTILEVEL || s == INPAINT_SCHED_CG_MULTIGRID;
}

// CG iterations per smoothing unless set: the fastest count on a 4K RGB frame
// with a 4 % mask, at rel-res 1e-3 and 1e-6 alike (measured over 1, 2, 4, 8).
constexpr int kCgSmoothMultilevel = 8, kCgSmoothMultigrid = 2;

// Validated options with defaults filled in (throws Fail on a bad value).
Opts resolve(const inpaint_opts* p);

// ---------------------------------------------------------------------------
// workspaces
// ---------------------------------------------------------------------------

struct Level {
  LevelView v;
  uint8_t* c = nullptr;
  float* b = nullptr;
  float* u[2] = {nullptr, nullptr};
  float* r = nullptr;
  float* contrib = nullptr;
  int* itot = nullptr;  // [C][nblk] local CG iterations per block, summed over a solve
  int* imax = nullptr;  // [C][nblk] their maximum (itot and imax are contiguous)
  int cur = 0;
  // Precision form, finest grid only: the V-cycle solves for a correction e of
  // the float32 iterate with 16-bit fields: e (double-buffered), its
  // right-hand side d (the float64 residual of u, rounded) and its residual rh.
  void* e[2] = {nullptr, nullptr};
  void* d = nullptr;
  void* rh = nullptr;
  int ecur = 0;
  bool ezero = true;  // e is zero (at the start of every V-cycle)
  // Deferred norm partials of this level's residual ([C][dstride]; dstride 0:
  // the level's norms are always reduced in the pass) and the number of
  // partials its latest writer left (0: the norm is in the workspace's snorm).
  double* dpart = nullptr;
  int dstride = 0;
  int npart = 0;
};

struct Key {
  int dev, W, H, C, B, o, coarsest, prec;
  bool operator==(const Key& k) const { return !(*this < k) && !(k < *this); }
  bool operator<(const Key& k) const {
    return std::tie(dev, W, H, C, B, o, coarsest, prec) <
           std::tie(k.dev, k.W, k.H, k.C, k.B, k.o, k.coarsest, k.prec);
  }
};

struct Workspace {
  Key key{};
  int L = 0;
  Level lv[kMaxLevels];
  void* base = nullptr;
  size_t bytes = 0;
  size_t maxtiles = 0;          // most pass workgroups over any level
  double* partials = nullptr;   // [C][maxtiles], kept unset between passes
  unsigned* counters = nullptr; // [C], kept at 0 between passes
  double* snorm = nullptr;  // [L][C]
  double* den = nullptr;    // [C]
  float* rho = nullptr;     // [C] rms of the reference residual (scale of 16-bit fields)
  double* relres = nullptr; // [C]
  int* active = nullptr;    // [C]
  int* status = nullptr;    // [4]
  int* checks = nullptr;    // [C] convergence tests run per channel
  unsigned long long* cgstat = nullptr;  // [L][C][3]: total, max, pixel-weighted local CG iterations
  std::vector<hipEvent_t> evpool;        // events for per-launch profiling
  // host-pointer staging (allocated on first use)
  void* stage_base = nullptr;
  float* f_dev = nullptr;
  uint8_t* m_dev = nullptr;
  float* o_dev = nullptr;
  // plain CG (comparison schedule, allocated on first use): two directions, A p,
  // and per channel r.r in two slots and p.q
  void* cg_base = nullptr;
  float* cg_p[2] = {nullptr, nullptr};
  float* cg_q = nullptr;
  double* cgs = nullptr;  // [3][C]
  // pinned readback
  void* host = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool busy = false;
  // cache bookkeeping: a serial number never reused by another workspace (it
  // keys cached batch plans), the last lease, and the lazily added buffers' sizes
  unsigned long long serial = 0, last_use = 0;
  size_t stage_bytes = 0, cg_bytes = 0;

  ~Workspace();
};

// Level sizes: halve with ceil until both sides are at most `coarsest`.
std::vector<std::pair<int, int>> level_sizes(int W, int H, int coarsest);

struct Lease {
  Workspace* ws = nullptr;
  Lease() = default;
  Lease(const Lease&) = delete;
  Lease& operator=(const Lease&) = delete;
  ~Lease();
};

// A workspace for key k: the grid hierarchy and all per-problem device state
// in one allocation (alloc = false: sizes only, nothing allocated).
std::unique_ptr<Workspace> create_workspace(const Key& k, bool alloc = true);
// Device bytes of create_workspace(k).
size_t workspace_bytes(const Key& k);
// A workspace for key k whose buffers live in caller-owned device memory at
// base (capacity bytes; nothing is allocated, the workspace never frees it):
// Fail (E_INVALID) when it needs more than capacity; its counters and norm
// partials are cleared on stream s.
std::unique_ptr<Workspace> bind_workspace(const Key& k, void* base, size_t capacity, hipStream_t s);
// Restore the state the kernels expect between passes (counters 0, norm
// partials unset, convergence-test counts 0), on stream s.
void clear_workspace_state(Workspace* ws, hipStream_t s);

// Lease a free workspace for (device, sizes, channels, block, overlap,
// coarsest side, precision), creating it on first use.  Idle workspaces stay
// cached for later calls within a byte limit (least recently used freed first).
void acquire(Lease& lease, int W, int H, int C, int B, int o, int coarsest, int prec = PREC_F32);
// Set the cache's byte limit (0: keep it), free idle workspaces above it, and
// return the bytes still cached.
size_t set_cache_limit(size_t limit);
// Device buffers for host-memory inputs and outputs (allocated on first use).
void ensure_staging(Workspace* ws);
// Buffers of the CG schedule (directions, A p, scalars); allocated once.
void ensure_cg(Workspace* ws);
bool is_device_ptr(const void* p);

// ---------------------------------------------------------------------------
// the cycle driver
// ---------------------------------------------------------------------------

struct Run {
  Workspace* ws;
  Opts o;
  hipStream_t s;
  int C;
  double tol;
  long oras_iters = 0;
  long block_solves = 0;
  long long finest_block_solves = 0;
  int top = 0;  // level whose b holds known values (a solution problem); coarser ones hold corrections
  // Level whose last ORAS update is left to the next prolongation from it
  // (its result is read by nothing else), per level.
  bool pend[kMaxLevels] = {};
  // CG schedule: slot of the current r.r in ws->cgs, buffer of the current direction
  int cg_slot = 0, cg_p = 0;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  size_t next_ev = 0;

  hipEvent_t pool_event() {
    if (next_ev == ws->evpool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      ws->evpool.push_back(e);
    }
    return ws->evpool[next_ev++];
  }

  // Launch through `fn`; on the finest grid with profiling on, bracket it by
  // two events on the same stream.
  template <class Fn>
  void timed(int cls, int level, Fn&& fn) {
    if (!o.profile || level != 0) {
      HIPCHK(fn());
      return;
    }
    hipEvent_t a = pool_event(), b = pool_event();
    HIPCHK(hipEventRecord(a, s));
    HIPCHK(fn());
    HIPCHK(hipEventRecord(b, s));
    recs.push_back({cls, a, b});
  }

  // Largest number of workgroup partials a block solve adds itself.
  static constexpr size_t kDeferMax = kDeferParts;

  // Norm of level l's residual written by a pass of writer_tiles workgroups.
  // The convergence test needs the full in-pass reduction; a norm that no
  // launch reads is skipped; on small grids the partials are left for the
  // block solve that reads the norm.
  NormOut norm(int l, bool check, size_t writer_tiles = (size_t)-1, bool need = true) {
    NormOut n{};
    Level& L = ws->lv[l];
    if (check) {
      n.mode = NORM_FULL;
      L.npart = 0;
    } else if (!need) {
      n.mode = NORM_NONE;
    } else if (L.dstride > 0 && writer_tiles <= (size_t)L.dstride) {
      n.mode = NORM_DEFER;
      n.dpart = L.dpart;
      n.dstride = L.dstride;
      L.npart = (int)writer_tiles;
    } else {
      n.mode = NORM_FULL;
      L.npart = 0;
    }
    n.partials = ws->partials;
    n.counter = ws->counters;
    n.status = ws->status;
    n.out = ws->snorm + (size_t)l * C;
    n.den = ws->den;
    n.relres = ws->relres;
    n.active = ws->active;
    n.checks = ws->checks;
    n.tol = tol;
    n.check = check ? 1 : 0;
    return n;
  }

  // Scales of 16-bit fields (kernels.h, Sc), relative to the reference
  // residual's rms rho: residuals and right-hand sides of level l carry the
  // integer stencil's factor 4^l; errors and corrections do not.  Fields of a
  // solution problem (iterate, known values: grey levels) are not scaled.
  static constexpr float kRes = 1e-3f, kErr = 1e-2f;
  static Sc sc_res(int l) { return Sc{kRes * std::ldexp(1.0f, 2 * l), 1}; }
  static Sc sc_err() { return Sc{kErr, 1}; }
  static Sc sc_one() { return Sc{1.0f, 0}; }
  int prec() const { return ws->key.prec; }
  // The finest grid runs the correction form (16-bit e on a float32 u): the
  // float16 form on a hierarchy of more than one level.  bfloat16's 8-bit
  // significand would bound each refinement step's contraction at ~4e-3 (a
  // third V-cycle at 4 % masks, measured), so in the bfloat16 form the finest
  // grid keeps float32 fields and only the coarser levels and the block
  // corrections are 16-bit.
  bool corr0() const { return ws->key.prec == PREC_F16 && ws->L > 1; }

  // Arguments of a pass over the finest grid's correction problem: iterate e,
  // right-hand side d, residual rh, all of the correction type.  The pass runs
  // `mode`, or `mode0` while e is still zero.
  PassArgs corr_args(int mode, int mode0) {
    Level& L = ws->lv[0];
    PassArgs a = pass_args(0);
    a.mode = L.ezero ? mode0 : mode;
    a.level0 = 0;
    a.solution = 0;
    a.s_u = sc_err();
    a.s_b = sc_res(0);
    a.s_r = sc_res(0);
    a.b = L.d;
    a.u_in = L.e[L.ecur];
    a.u_out = L.e[L.ecur ^ 1];
    a.r = L.rh;
    L.ecur ^= 1;
    L.ezero = false;
    return a;
  }

  PassArgs pass_args(int l) const {
    const Level& L = ws->lv[l];
    PassArgs a{};
    a.lv = L.v;
    a.prec = prec();
    a.level0 = l == 0;
    a.solution = l == top ? 1 : 0;
    a.rho = ws->rho;
    a.s_u = a.solution ? sc_one() : sc_err();
    a.s_b = a.solution ? sc_one() : sc_res(l);
    a.s_r = sc_res(l);
    a.s_contrib = sc_err();
    a.s_cr = sc_res(l + 1);
    a.c = L.c;
    a.b = L.b;
    a.u_in = L.u[L.cur];
    a.u_out = L.u[L.cur ^ 1];
    a.r = L.r;
    a.contrib = L.contrib;
    a.active = ws->active;
    return a;
  }

  // ---- argument builders: each returns the arguments of one launch and
  // advances the host-side state (which buffer holds the iterate, counters)
  // exactly as running that launch would.

  PassArgs make_residual(int l, bool check) {
    PassArgs a = pass_args(l);
    a.mode = PASS_RES;
    a.u_out = nullptr;
    a.norm = norm(l, check, pass_tiles(ws->lv[l].v));
    if (l == 0 && corr0()) {
      // the residual of u is the right-hand side of the next correction problem
      a.r = ws->lv[0].d;
      a.r_tc = 1;
      ws->lv[0].ezero = true;
    }
    return a;
  }

  BlockArgs make_block(int l) {
    Level& L = ws->lv[l];
    BlockArgs b{};
    b.lv = L.v;
    b.prec = prec();
    b.level0 = l == 0;
    b.rho = ws->rho;
    b.s_r = sc_res(l);
    b.s_contrib = sc_err();
    b.c = L.c;
    b.r = L.r;
    if (l == 0 && corr0()) {
      b.level0 = 0;
      b.r = L.ezero ? L.d : L.rh;  // while e = 0 its residual is d
    }
    b.snorm = L.npart ? L.dpart : ws->snorm + (size_t)l * C;
    b.npart = L.npart;
    b.pstride = L.dstride;
    b.contrib = L.contrib;
    b.gamma = o.gamma;
    b.tau = o.tau;
    b.inv_o1 = 1.0f / (float)(L.v.o - 1);
    b.inv_area = 1.0 / ((double)L.v.W * (double)L.v.H);
    b.maxit = o.maxit;
    b.active = ws->active;
    b.itot = o.profile ? L.itot : nullptr;
    b.imax = o.profile ? L.imax : nullptr;
    return b;
  }

  // The update half of an ORAS iteration.  With rest, it also restricts the
  // new residual to level l + 1 (the last pre-smoothing of a V-cycle).  need:
  // some later launch reads the norm this pass writes.
  PassArgs make_update(int l, bool check, bool rest, bool need = true) {
    Level& L = ws->lv[l];
    const bool corr = l == 0 && corr0();
    if (corr && check) fail(INPAINT_E_DEVICE, "a correction update cannot test convergence");
    PassArgs a = corr ? corr_args(PASS_UPD, PASS_UPD0) : pass_args(l);
    if (!corr) a.mode = PASS_UPD;
    const size_t tiles = pass_tiles(L.v);
    if (!rest) a.norm = norm(l, check, tiles, need);
    if (rest) {
      Level& Cl = ws->lv[l + 1];
      a.rest = 1;
      a.clv = Cl.v;
      a.cc = Cl.c;
      a.bc = Cl.b;
      a.uc0 = Cl.u[Cl.cur];
      a.rc = Cl.r;
      // the coarsest grid's solve does not read the norm
      a.norm = norm(l + 1, false, tiles, need && l + 1 < ws->L - 1);
    }
    if (!corr) L.cur ^= 1;
    ++oras_iters;
    block_solves += (long)L.v.nbx * L.v.nby * C;
    if (l == 0) finest_block_solves += (long long)L.v.nbx * L.v.nby * C;
    return a;
  }

  // The update half of an ORAS iteration on level l >= 1 whose new iterate
  // only the next prolongation from level l reads (no residual, no norm):
  // that prolongation adds the block corrections itself.
  void defer_update(int l) {
    Level& L = ws->lv[l];
    if (l == 0 || pend[l]) fail(INPAINT_E_DEVICE, "update cannot be deferred");
    pend[l] = true;
    ++oras_iters;
    block_solves += (long)L.v.nbx * L.v.nby * C;
  }
  bool pending() const {
    for (bool p : pend)
      if (p) return true;
    return false;
  }

  PassArgs make_prolong(int l, int mode, bool check, bool need = true) {
    Level& L = ws->lv[l];
    const Level& Lc = ws->lv[l + 1];
    const bool corr = l == 0 && corr0() && mode == PASS_PCORR;
    if (corr && check) fail(INPAINT_E_DEVICE, "a correction pass cannot test convergence");
    PassArgs a = corr ? corr_args(PASS_PCORR, PASS_PCORR0) : pass_args(l);
    if (!corr) a.mode = mode;
    if (l == 0 && corr0() && mode == PASS_PSOL) {
      a.r = L.d;
      a.r_tc = 1;
      L.ezero = true;
    }
    a.uc = Lc.u[Lc.cur];
    if (pend[l + 1]) {
      a.ccontrib = Lc.contrib;
      a.clv = Lc.v;
      pend[l + 1] = false;
    }
    // the coarse field is a solution in the cascade and a correction in a V-cycle
    a.s_uc = mode == PASS_PSOL ? sc_one() : sc_err();
    a.Wc = Lc.v.W;
    a.Hc = Lc.v.H;
    a.Pc = Lc.v.P;
    a.planec = Lc.v.plane;
    a.norm = norm(l, check, pass_tiles(L.v), need);
    if (!corr) L.cur ^= 1;
    return a;
  }

  // Precision form, finest grid: u += e (+ the block corrections of the ORAS
  // iteration whose block solves just ran, when `blocks`), then the float64
  // residual of the new u, its norm and the convergence test; the residual,
  // rounded, is the right-hand side d of the next correction problem.
  PassArgs make_final(bool check, bool blocks) {
    Level& L = ws->lv[0];
    PassArgs a = pass_args(0);
    a.mode = blocks ? PASS_FIN : PASS_FIN0;
    a.e_add = L.ezero ? nullptr : L.e[L.ecur];
    a.s_e = sc_err();
    if (!blocks) a.contrib = nullptr;
    a.r = L.d;
    a.r_tc = 1;
    a.norm = norm(0, check);
    L.cur ^= 1;
    L.ezero = true;
    if (blocks) {
      ++oras_iters;
      block_solves += (long)L.v.nbx * L.v.nby * C;
      finest_block_solves += (long long)L.v.nbx * L.v.nby * C;
    }
    return a;
  }

  // ---- plain CG (comparison schedules): on the finest grid alone, or as the
  // smoother of every level in the multilevel and multigrid counterparts.
  // Each pass that (re)computes r on a level puts r.r in the current slot, and
  // the smoothing that follows starts its recurrence there.

  // A full in-pass reduction of level l into `out` (with the convergence test
  // when check).
  NormOut cg_norm(int l, double* out, bool check = false) {
    NormOut n = norm(l, check);
    n.mode = NORM_FULL;
    n.out = out;
    return n;
  }
  double* cg_rr() const { return ws->cgs + (size_t)cg_slot * C; }

  // Float64 true residual r = b - A x of level l (with the convergence test on
  // the finest grid).  It replaces the recurrence's r of the same iterate, and
  // its norm replaces that r.r in the current slot (the iteration does not
  // advance: the next direction's beta divides by the r.r of the previous
  // iterate).
  PassArgs make_cg_residual(int l = 0, bool check = true) {
    PassArgs a = make_residual(l, check);
    a.norm = cg_norm(l, cg_rr(), check);
    return a;
  }
  // A prolongation (PSOL in the cascade, PCORR in a V-cycle) whose residual
  // norm starts the smoothing of level l.
  PassArgs make_cg_prolong(int l, int mode, bool check) {
    PassArgs a = make_prolong(l, mode, check);
    a.norm = cg_norm(l, cg_rr(), check);
    return a;
  }
  // The float64 residual of level l after its pre-smoothing (no norm), and its
  // restriction to level l + 1, whose norm starts the smoothing there.
  PassArgs make_cg_pre_residual(int l) {
    PassArgs a = make_residual(l, false);
    a.norm.mode = NORM_NONE;
    Level& L = ws->lv[l];
    L.npart = 0;
    return a;
  }
  RestrictArgs make_cg_restrict(int l) {
    RestrictArgs a = make_restrict(l);
    a.norm = cg_norm(l + 1, cg_rr());
    return a;
  }
  CgArgs cg_args(int l) const {
    const Level& L = ws->lv[l];
    CgArgs a{};
    a.lv = L.v;
    a.c = L.c;
    a.x = L.u[L.cur];
    a.r = L.r;
    a.q = ws->cg_q;
    a.active = ws->active;
    return a;
  }
  // p = r + beta p (p = r when first), q = A p, p.q
  CgArgs make_cg_dir(int l, bool first) {
    CgArgs a = cg_args(l);
    a.p_in = ws->cg_p[cg_p];
    a.p_out = ws->cg_p[cg_p ^ 1];
    cg_p ^= 1;
    a.rho = cg_rr();
    a.rho_old = ws->cgs + (size_t)(cg_slot ^ 1) * C;
    a.first = first ? 1 : 0;
    a.norm = cg_norm(l, ws->cgs + 2 * (size_t)C);
    return a;
  }
  // x += alpha p, r -= alpha q, r.r into the next slot
  CgArgs make_cg_step(int l) {
    CgArgs a = cg_args(l);
    a.p_in = ws->cg_p[cg_p];
    a.rho = cg_rr();
    a.pq = ws->cgs + 2 * (size_t)C;
    cg_slot ^= 1;
    a.norm = cg_norm(l, cg_rr());
    ++oras_iters;
    return a;
  }

  RestrictArgs make_restrict(int l) {
    const Level& F = ws->lv[l];
    Level& Cl = ws->lv[l + 1];
    RestrictArgs a{};
    a.fl = F.v;
    a.cl = Cl.v;
    a.prec = prec();
    a.level0 = l == 0;
    a.rf = F.r;
    if (l == 0 && corr0()) {
      // pre-smoothing is off: e = 0, so the residual to restrict is d
      a.level0 = 0;
      a.rf = F.d;
    }
    a.cc = Cl.c;
    a.bc = Cl.b;
    a.uc = Cl.u[Cl.cur];
    a.rc = Cl.r;
    a.norm = norm(l + 1, false, pass_tiles(Cl.v), l + 1 < ws->L - 1);
    a.active = ws->active;
    a.rho = ws->rho;
    a.s_rf = sc_res(l);
    a.s_cr = sc_res(l + 1);
    return a;
  }

  CoarseArgs make_coarse(int l, bool init) {
    Level& L = ws->lv[l];
    CoarseArgs a{};
    a.lv = L.v;
    a.prec = prec();
    a.level0 = l == 0;
    a.rho = ws->rho;
    const bool sol = l == top;
    a.s_b = sol ? sc_one() : sc_res(l);
    a.s_u = sol ? sc_one() : sc_err();
    a.c = L.c;
    a.b = L.b;
    a.u = L.u[L.cur];
    a.init = init ? 1 : 0;
    a.rel_tol = o.coarse_tau;
    a.maxit = o.coarse_maxit;
    a.active = ws->active;
    return a;
  }

  // ---- single-problem launches

  void residual(int l, bool check) {
    const PassArgs a = make_residual(l, check);
    timed(INPAINT_K_RESIDUAL, l, [&] { return launch_pass(a.mode, a, C, s); });
  }

  void oras(int l, bool check, bool rest = false) {
    const BlockArgs b = make_block(l);
    timed(INPAINT_K_BLOCK_SOLVE, l, [&] { return launch_block_solve(b, C, s); });
    const PassArgs a = make_update(l, check, rest);
    timed(INPAINT_K_UPDATE, l, [&] { return launch_pass(a.mode, a, C, s); });
  }

  void prolong(int l, int mode, bool check) {
    const PassArgs a = make_prolong(l, mode, check);
    timed(INPAINT_K_PROLONG, l, [&] { return launch_pass(a.mode, a, C, s); });
  }

  void restrict_to(int l) {
    const RestrictArgs a = make_restrict(l);
    timed(INPAINT_K_RESTRICT, l, [&] { return launch_restrict(a, C, s); });
  }

  void coarse(int l, bool init) {
    const CoarseArgs a = make_coarse(l, init);
    timed(INPAINT_K_COARSE, l, [&] { return launch_coarse_solve(a, C, s); });
  }
};


// Stage (f, mask) into level 0 and build the hierarchy; returns after the
// input checks have been read back.
void prepare(Run& R, const float* f_d, const uint8_t* m_d, bool hierarchy, bool write_u);
void check_dims(const void* a, const void* b, int W, int H, int C);
// Throws Fail (E_INVALID) for an image whose fields or block corrections
// would overflow the kernels' 32-bit offsets for block side B and overlap o.
void check_geometry(int W, int H, int B, int o);
bool overlap(const void* a, size_t na, const void* b, size_t nb);

}  // namespace inpaint
