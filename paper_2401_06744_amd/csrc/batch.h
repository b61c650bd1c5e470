// Batched execution: plans of batched launches over many problems, and the
// per-problem state of a batch.  Internal; shared by the batched and the
// serving entry points.
#pragma once

#include <array>
#include <memory>
#include <string>
#include <vector>

#include "driver.h"

namespace inpaint {

enum StepKind : int {
  S_RESET,
  S_STAGE,
  S_RHS,
  S_PASS,
  S_RESTRICT,
  S_BLOCK,
  S_COARSE,
  S_OUTPUT,
  S_GATHER,
  S_CG_DIR,
  S_CG_STEP,
  S_WARM,
};

// One batched launch: n argument structs and n + 1 work offsets, stored at
// byte offsets `args` and `start` of the plan's buffer.  `f32` selects the
// kernel variant whose level fields are float32 (the finest grid's solution
// fields); `level` is the grid level the launch works on (-1: none).
struct Step {
  int kind, mode, f32, level, n;
  unsigned total;
  size_t args, start;
};

// A sequence of batched launches whose arguments live in one device buffer.
struct Plan {
  std::vector<Step> steps;
  std::vector<unsigned char> host;  // argument arrays and offsets, packed
  unsigned char* dev = nullptr;     // device copy of `host` (owned by the batch context)
  // per member of the batch: what one run of the plan adds to its ORAS
  // iterations, block solves and finest-grid block solves, and which level-0
  // buffer holds its iterate afterwards
  std::vector<std::array<long long, 3>> delta;
  std::vector<int> cur0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  void begin(int kind, int mode = 0, int level = -1);
  // Append one problem's arguments; f32 (if >= 0) is the field type of its
  // launch variant, which every problem of a launch must share.
  template <class T>
  void add(const T& a, unsigned work, int f32 = -1) {
    if (f32 >= 0) {
      if (open.f32 < 0)
        open.f32 = f32;
      else if (open.f32 != f32)
        fail(INPAINT_E_DEVICE, "problems of one batched launch need different kernel variants");
    }
    const size_t at = pend.size();
    pend.resize(at + sizeof(T));
    std::memcpy(pend.data() + at, &a, sizeof(T));
    open.n += 1;
    pstart.push_back(pstart.back() + work);
  }
  // A pass launch: the problems must also share the pass mode.
  void add_pass(const PassArgs& a, unsigned work) {
    if (open.mode < 0)
      open.mode = a.mode;
    else if (open.mode != a.mode)
      fail(INPAINT_E_DEVICE, "problems of one batched launch need different pass modes");
    add(a, work, a.level0);
  }
  void end();
  void clear();
  Plan() = default;
  Plan(const Plan&) = delete;
  Plan& operator=(const Plan&) = delete;
  ~Plan();

 private:
  size_t append(const void* p, size_t n);
  Step open{};
  std::vector<unsigned char> pend;
  std::vector<unsigned> pstart;
};

// Per-launch timing of the finest-grid launches (single solves with
// opts.profile): HIP events recorded around each such launch on its stream.
struct Prof {
  std::vector<hipEvent_t>* pool = nullptr;  // reused events (owned by the workspace)
  size_t next = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipEvent_t event();
};

// Enqueue every launch of a plan (plan.dev must be set).
hipError_t issue(const Plan& P, int prec, int B, hipStream_t s, Prof* prof = nullptr);

// One problem of a batch.
struct Member {
  int idx = 0;   // position in the caller's array
  int slot = 0;  // slot of its flag block (kFlagInts ints) in the gathered flag array
  int W = 0, H = 0, C = 0;
  Lease lease;
  Workspace* ws = nullptr;
  std::unique_ptr<Run> R;
  const float* f_d = nullptr;
  const uint8_t* m_d = nullptr;
  float* o_d = nullptr;  // device output (the caller's, or staging)
  float* out = nullptr;  // the caller's output
  bool out_host = false;
  int status = INPAINT_OK;
  std::string msg;
  std::vector<int> final_cur;  // per channel: level-0 buffer of the final iterate, -1 while running
  std::vector<double> rel;
  int cycles = 0;
  bool done = false;
  long long oras = 0, blocks = 0, finest_blocks = 0;
  int Lc() const { return ws->L - 1; }
};

// Plan builders.  Each walks the members in lockstep by level and calls their
// Run's argument builders in the order a solve of that member alone launches.
// Prepare: reset flags, stage (f, mask) into level 0 with the reference
// residual, coarse masks and known values level by level, gather the flags.
void build_prepare(Plan& P, const std::vector<Member*>& ms, const Opts& o, int* flags_dev);
// The coarse-to-fine initial guess (Section 4.2); for the CG schedules the
// first CG step (plain CG) or the cascade with CG smoothing.
void build_cascade(Plan& P, const std::vector<Member*>& ms, const Opts& o);
// One V-cycle on the finest grid (one finest ORAS iteration for the
// multilevel and single-level schedules; 8 CG iterations and a convergence
// test for plain and multilevel CG; a V-cycle with CG smoothing for
// multigrid CG).
void build_cycle(Plan& P, const std::vector<Member*>& ms, const Opts& o);
void build_output(Plan& P, const std::vector<Member*>& ms);
// Copy of each member's flag block to flags_dev + kFlagInts * member.slot.
void add_gather(Plan& P, const std::vector<Member*>& ms, int* flags_dev);

// Build a plan with `body` and record, per member, what one run of it adds to
// the member's counters and which level-0 buffer holds the iterate afterwards.
template <class Body>
void build(Plan& P, const std::vector<Member*>& ms, Body&& body) {
  std::vector<std::array<long long, 3>> before;
  for (Member* m : ms) before.push_back({m->R->oras_iters, m->R->block_solves, m->R->finest_block_solves});
  body();
  for (Member* m : ms)
    if (m->R->pending()) fail(INPAINT_E_DEVICE, "a deferred update has no prolongation to take it");
  P.delta.clear();
  P.cur0.clear();
  for (size_t i = 0; i < ms.size(); ++i) {
    const Run& R = *ms[i]->R;
    P.delta.push_back({R.oras_iters - before[i][0], R.block_solves - before[i][1],
                       R.finest_block_solves - before[i][2]});
    P.cur0.push_back(ms[i]->ws->lv[0].cur);
  }
}

// Host-side iteration state of the members (which buffer of each level holds
// the iterate, CG slots): cycle plans alternate until it repeats.
std::vector<int> level_state(const std::vector<Member*>& ms);

// Copy the plans' argument arrays into one device buffer owned by `*buf`
// (grown as needed) and point each plan at its part.
void upload(std::vector<Plan*> plans, unsigned char** buf, size_t* cap, hipStream_t s);

// Set up member m for problem p on workspace ws: stage host inputs, pick the
// output buffer.  m.idx and m.slot are set by the caller.
void init_member(Member& m, const inpaint_problem& p, Workspace* ws, const Opts& o, double tol,
                 hipStream_t s);
// Throws Fail (E_INVALID) for a bad problem (including sizes the kernels
// cannot address with options o); i >= 0 names it in the message.
void validate_problem(const inpaint_problem& p, int i, const Opts& o);
// Input checks read back after a prepare plan; sets m->status on rejection.
void check_prepared(const int* flags_host, Member* m);
// Apply gathered flags after plan P ran over ms; returns true when all are done.
bool apply_flags(const int* flags_host, const std::vector<Member*>& ms, const Plan& P);
// Apply gathered flags after the plans seq (the cascade, then cycle plans in
// issue order) ran over ms: each channel's count of convergence tests names
// the plan it stopped in.  Sets final buffers, counters and cycle counts;
// returns true when all are done.
bool apply_counted(const int* flags_host, const std::vector<Member*>& ms,
                   const std::vector<const Plan*>& seq);
// Back to the state init_member left (before a repeated solve).
void reset_member(Member* m);
// Add one run of P to the counters of the members still running.
void account(const std::vector<Member*>& ms, const Plan& P);
// After the last plan: final buffers of unfinished channels and the status.
void finish_member(Member* m, int last_cur0);
void fill_stats(const Member* m, inpaint_stats& st);

// Solve the members together (prepare, cascade, V-cycles, output), on the
// stream s, and return after every result is in place; statuses, iteration
// state and statistics are left in the members.  With prof (single solves
// with opts.profile) every finest-grid launch is timed and nothing is replayed
// from a graph.  Returns the device time in ms.
float run_batch(const std::vector<Member*>& all, const Opts& o, double tol, hipStream_t s,
                Prof* prof);

// Device resources of a batch, cached across calls with the same workspaces,
// options and tolerance.
struct BatchCtx {
  std::string key;
  std::string live_key;  // which members the cached plans were built for
  int dev_id = 0, n = 0;
  Plan cascade;
  Plan cycle[2];  // cycle plans alternate when a V-cycle flips the iterate buffers
  int ncycle = 0;
  // V-cycles the last solve in this context needed (all members converged);
  // 0: wait for the input checks and test convergence after every plan
  int expect = 0;
  unsigned char* plan_dev = nullptr;
  size_t plan_cap = 0;
  unsigned char* call_dev = nullptr;  // per-call plans (prepare, output)
  size_t call_cap = 0;
  int* flags_dev = nullptr;   // [n][kFlagInts] gathered flag blocks
  int* flags_host = nullptr;  // pinned copy
  hipStream_t cap = nullptr;  // capture stream
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  ~BatchCtx();
};

}  // namespace inpaint
