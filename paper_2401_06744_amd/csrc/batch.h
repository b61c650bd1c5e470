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
  S_MASK,
  S_RHS,
  S_PASS,
  S_RESTRICT,
  S_BLOCK,
  S_COARSE,
  S_OUTPUT,
  S_GATHER,
};

// One batched launch: n argument structs and n + 1 work offsets, stored at
// byte offsets `args` and `start` of the plan's buffer.
struct Step {
  int kind, mode, level0, n;
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

  void begin(int kind, int mode = 0, int level0 = 0);
  template <class T>
  void add(const T& a, unsigned work) {
    const size_t at = pend.size();
    pend.resize(at + sizeof(T));
    std::memcpy(pend.data() + at, &a, sizeof(T));
    open.n += 1;
    pstart.push_back(pstart.back() + work);
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

// Enqueue every launch of a plan (plan.dev must be set).
hipError_t issue(const Plan& P, int prec, int B, hipStream_t s);

// One problem of a batch.
struct Member {
  int idx = 0;   // position in the caller's array
  int slot = 0;  // 64-byte slot of its flags in the gathered flag array
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

// Device resources of a batch, cached across calls with the same workspaces,
// options and tolerance.
struct BatchCtx {
  std::string key;
  std::string live_key;  // which members the cached plans were built for
  int dev_id = 0, n = 0;
  Plan cascade;
  Plan cycle[2];  // cycle plans alternate when a V-cycle flips the iterate buffers
  int ncycle = 0;
  unsigned char* plan_dev = nullptr;
  size_t plan_cap = 0;
  unsigned char* call_dev = nullptr;  // per-call plans (prepare, output)
  size_t call_cap = 0;
  int* flags_dev = nullptr;   // [n][16] gathered flag blocks
  int* flags_host = nullptr;  // pinned copy
  hipStream_t cap = nullptr;  // capture stream
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  ~BatchCtx();
};

}  // namespace inpaint
