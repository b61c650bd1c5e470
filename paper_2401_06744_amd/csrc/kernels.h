// Internal declarations shared by the gfx950 kernels and the host driver.
// Not part of the public ABI (see include/inpaint.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace inpaint {

constexpr int kMaxChannels = 4;
constexpr int kCounterGroups = 64;
constexpr int kCounterLines = kCounterGroups + 1;
constexpr int kMaxLevels = 24;

// Tile of the grid passes: 64 columns x 32 rows, 256 threads (8 rows each).
constexpr int kTileW = 64;
constexpr int kTileH = 32;
// Bit pattern of an unset norm partial: a NaN with a payload no arithmetic
// produces (partials may be negative: CG's p.q), compared bit for bit.
constexpr unsigned long long kUnsetPartialBits = 0xFFF7C0FFEE5E7A11ull;
inline double unset_partial() { return __builtin_bit_cast(double, kUnsetPartialBits); }

// Ints per flag block of a problem: relres[4] doubles, active[4], status[4],
// checks[4] ints, then kKnownWords "a known pixel was seen" words (status[8]
// .. status[8 + kKnownWords - 1]; the staging writes 2 into the word of its XCD
// with a plain store, so that no word is shared by all of a launch's
// workgroups), spare.  One block is copied to the host per poll.
constexpr int kFlagInts = 32;
constexpr int kKnownWords = 8;
constexpr int kKnownAt = 8;  // offset of the known words from status[0]
// Input checks of a flag block (its status[0] .. status[kKnownAt + kKnownWords - 1]):
// bit 1 a known pixel with non-finite f, bit 2 some known pixel exists.
inline int input_checks(const int* status) {
  int st = status[0] & 1;
  for (int i = 0; i < kKnownWords; ++i) st |= status[kKnownAt + i] & 2;
  return st | (status[0] & 2);
}
// Most norm partials a block solve adds up itself (deferred norms).
constexpr int kDeferParts = 256;

// Storage precision of the correction fields (the weighted block corrections
// on every level and every field of the coarser levels).  The finest grid's
// iterate, known values and residual are always float32.
enum Prec : int { PREC_F32 = 0, PREC_F16 = 1, PREC_BF16 = 2 };

// One grid level as the kernels see it.  Fields are planar per channel with a
// padded row pitch P (elements); one plane holds H*P elements.
struct LevelView {
  int W, H, P;
  size_t plane;
  int nbx, nby;  // ORAS blocks along x and y
  int B, o;      // block side and overlap (stride B - o)
};

// Scale of a field stored in 16 bits: stored = value / (f * (rel ? rho[ch] : 1)).
// rho[ch] is the rms of the channel's reference residual, so that residuals
// and corrections keep their magnitudes inside the float16 range at every
// accuracy from the first cycle to the tolerance.  Ignored for float32 fields.
struct Sc {
  float f;
  int rel;
};

// Per-channel norm reduction of a grid pass.
//   NORM_FULL:  every workgroup publishes its partial sum and bumps a
//               per-channel counter; the workgroup that arrives last adds all
//               partials in a fixed order and writes the norm (and the
//               convergence test) - needed on large grids and for the test.
//   NORM_DEFER: every workgroup stores its partial sum at dpart[ch * dstride +
//               tile] and nothing more; the block solve that consumes the norm
//               adds the partials itself (cheap on small grids, and it saves
//               the pass the latency of the cross-workgroup reduction).
//   NORM_NONE:  nobody reads this norm.
enum NormMode : int { NORM_FULL = 0, NORM_DEFER = 1, NORM_NONE = 2 };

struct NormOut {
  int mode;
  double* dpart;      // NORM_DEFER: [C][dstride]
  int dstride;
  double* partials;   // [C][ntiles], every entry kUnsetPartial between passes
  unsigned* counter;  // [C][kCounterLines][32]: 64 group counters + 1 total, one
                      // 128-byte line each, all 0 between passes
  int* status;        // bit 2 (value 4) set if a partial never arrived
  double* out;        // [C] squared norm of the residual written by the pass
  // Optional convergence test on the finest grid (check != 0):
  const double* den;  // [C] squared norm of the reference residual
  double* relres;     // [C] sqrt(out / den)
  int* active;        // [C] set to 0 once relres <= tol
  int* checks;        // [C] number of tests run (optional)
  double tol;
  int check;
  // Optional (stage only): rho[ch] = sqrt(out[ch] * inv_n), the rms of the
  // reference residual, floored to a tiny positive value.
  float* rho;
  double inv_n;
};

enum PassMode : int {
  PASS_RES = 0,     // u_new = u_in (residual only; u_out unused)
  PASS_UPD = 1,     // u_new = u_in + sum of weighted block corrections
  PASS_PSOL = 2,    // u_new = mask ? b : P u_c   (cascade prolongation)
  PASS_PCORR = 3,   // u_new = u_in + (mask ? 0 : P u_c)   (coarse-grid correction)
  // the precision form's finest grid (a 16-bit correction e of a float32 u):
  PASS_UPD0 = 4,    // as PASS_UPD with u_in = 0 (not read)
  PASS_FIN = 5,     // u_new = u_in + (e + sum of weighted block corrections), r of type prec
  PASS_FIN0 = 6,    // u_new = u_in + e, r of type prec
  PASS_PCORR0 = 7,  // as PASS_PCORR with u_in = 0 (not read)
};
constexpr int kPassModes = 8;

// The launch's own iterate, known values / right-hand side and residual are
// float32 when level0 = 1 (the finest grid's solution fields) and of the
// correction type `prec` otherwise; corrections, the coarse field and the fused
// restriction's outputs are always of type `prec`.
struct PassArgs {
  LevelView lv;
  int prec, level0;
  // 1 when b is 0 at every unknown pixel (the level holds a solution problem,
  // not a correction problem); b is then not read by PASS_UPD/PSOL/PCORR.
  int solution;
  const uint8_t* c;
  const void* b;
  const void* u_in;
  void* u_out;
  void* r;
  const void* contrib;   // PASS_UPD, UPD0, FIN: [C][nby*nbx][B][B]
  const void* uc;        // PASS_PSOL/PCORR: coarse field [C][Hc][Pc]
  int Wc, Hc, Pc;
  size_t planec;
  // PASS_PSOL/PCORR: when not null, the coarse field still lacks the update of
  // its last ORAS iteration: the prolongation reads uc + the weighted block
  // corrections ccontrib of the coarse level (geometry clv, scale s_contrib),
  // rounded to the coarse field's type as the update pass would have stored it.
  const void* ccontrib;
  NormOut norm;
  const int* active;     // [C] or nullptr: skip channels already converged
  // PASS_UPD with rest != 0: instead of writing the fine residual and its norm,
  // restrict it (Sections 4.1, 4.4) to the coarse level: write bc = rc = the
  // coarse right-hand side, uc0 = 0, and reduce the coarse norm into `norm`.
  int rest;
  LevelView clv;
  const uint8_t* cc;
  void* bc;
  void* uc0;
  void* rc;
  const float* rho;      // [C]
  Sc s_u, s_b, s_r, s_contrib, s_uc, s_cr;  // s_cr: coarse b and r of the restriction
  int mode;              // the PassMode this launch runs (all problems of a launch share it)
  const void* e_add;     // PASS_FIN, PASS_FIN0: the correction e (type prec, scale s_e)
  Sc s_e;
  int r_tc;              // PASS_PSOL, PASS_RES: the residual r is stored with type prec
};

struct BlockArgs {
  LevelView lv;
  int prec, level0;
  const uint8_t* c;
  const void* r;          // residual [C][H][P] (float32 on the finest grid)
  const double* snorm;    // [C] squared global residual norm, or (npart > 0) the sum of
  int npart, pstride;     // its npart partials at snorm[ch * pstride + i]
  void* contrib;          // [C][nby*nbx][B][B] weighted corrections D_i v_i (type prec)
  float gamma, tau;
  int maxit;
  const int* active;
  int* itot;              // [C][nby*nbx] running total of local CG iterations per block,
  int* imax;              // and the running maximum; both nullptr to skip
  const float* rho;
  Sc s_r, s_contrib;
  float inv_o1;           // 1 / (overlap - 1): slope of the partition-of-unity weights
  double inv_area;        // 1 / (W * H) of the level
};

struct CoarseArgs {
  LevelView lv;  // a single block covers the level
  int prec, level0;
  const uint8_t* c;
  const void* b;
  void* u;       // in/out
  int init;      // 1: start from u = C b;  0: continue from u
  float rel_tol; // stop when ||rho||^2 <= rel_tol * ||rho_0||^2
  int maxit;
  const int* active;
  const float* rho;
  Sc s_b, s_u;
};

struct RestrictArgs {
  LevelView fl, cl;
  int prec, level0;       // level0: the fine level is the finest grid (float32 residual)
  const void* rf;
  const uint8_t* cc;
  void* bc;
  void* uc;
  void* rc;
  NormOut norm;
  const int* active;
  const float* rho;
  Sc s_rf, s_cr;
};

struct StageArgs {
  const float* f;
  const uint8_t* mask;
  int W, H, Pf, C;
  LevelView lv;
  uint8_t* c;
  float* b;
  float* u;      // nullptr: not written
  int* status;
  NormOut den;
};

struct RhsArgs {
  LevelView fl, cl;
  const uint8_t* cf;
  const void* bf;
  uint8_t* cc;  // written: the coarse mask
  void* bc;
  int C, naive;
};

// Plain conjugate gradients on the finest grid (the comparison schedule): the
// direction pass p = r + beta p, q = A p and p.q, then the step pass
// x += alpha p, r -= alpha q and r.r.  A is the masked 5-point operator
// (identity rows at known pixels, where r, p and q are 0); scalars are
// float64 per channel, fields float32.
struct CgArgs {
  LevelView lv;
  const uint8_t* c;
  float* x;
  float* r;
  const float* p_in;      // direction pass: previous direction (not read when first); step: p
  float* p_out;           // direction pass: new direction
  float* q;               // A p
  const double* rho;      // [C] current r.r
  const double* rho_old;  // [C] previous r.r (direction pass)
  const double* pq;       // [C] p.q (step pass)
  int first;              // direction pass: p = r
  const int* active;
  NormOut norm;           // p.q (direction pass) or r.r (step pass)
};

// Output of one problem.  flags null: u[ch] is channel ch's final iterate.
// flags set (the output issued before the host has read the convergence
// tests): u[0], u[1] are the two level-0 iterate buffers and each channel's is
// chosen on the device from the problem's flag block: a channel that stopped
// after its k-th test (k = 1 the cascade, k > 1 cycle plan (k - 2) % ncycle)
// ends in buffer cur[0] resp. cur[1 + (k - 2) % ncycle]; a channel still
// iterating, a k outside 1..nplan, or a problem whose input checks failed is
// not written.
struct OutputArgs {
  LevelView lv;
  const uint8_t* c;
  const float* b;
  const float* u[kMaxChannels];
  float* out;
  int Pout, C;
  const int* flags;
  int nplan, ncycle;
  int cur[3];
  // reference residual norms [C] (nullptr: not read): a channel whose
  // ||b - A C f|| is 0 is solved exactly by C f, which is written
  const double* den;
};

// Initial guess of a warm-started solve on the finest grid: u = known ? b :
// src, with src the caller's planar buffer [C][H][Psrc].
struct WarmArgs {
  LevelView lv;
  const uint8_t* c;
  const float* b;
  float* u;
  const float* src;
  int Psrc, C;
};

// Work items (workgroups) of one problem in each kernel; a batched launch
// gives problem p the global items [start[p], start[p + 1]).
unsigned work_stage(const StageArgs& a);
unsigned work_rhs(const RhsArgs& a);
unsigned work_pass(const PassArgs& a, int C);
unsigned work_restrict(const RestrictArgs& a, int C);
unsigned work_block(const BlockArgs& a, int C);
unsigned work_coarse(const CoarseArgs& a, int C);
unsigned work_output(const OutputArgs& a);
unsigned work_warm(const WarmArgs& a);

// Batched launches: `args` (device) holds n argument structs, `start` (device)
// n + 1 offsets, `total` = start[n].  Every problem shares the kernel variant:
// mode, precision, level0 (passes) and block side (block/coarse solves); the
// channel count may differ between problems.
hipError_t launch_stage_b(const StageArgs* args, const unsigned* start, int n, unsigned total,
                          hipStream_t s);
hipError_t launch_rhs_b(const RhsArgs* args, const unsigned* start, int n, unsigned total, int prec,
                        int fine_f32, hipStream_t s);
hipError_t launch_pass_b(int mode, const PassArgs* args, const unsigned* start, int n,
                         unsigned total, int prec, int level0, hipStream_t s);
hipError_t launch_restrict_b(const RestrictArgs* args, const unsigned* start, int n, unsigned total,
                             int prec, int level0, hipStream_t s);
hipError_t launch_block_b(const BlockArgs* args, const unsigned* start, int n, unsigned total,
                          int prec, int level0, int B, hipStream_t s);
hipError_t launch_coarse_b(const CoarseArgs* args, const unsigned* start, int n, unsigned total,
                           int prec, int level0, int B, hipStream_t s);
hipError_t launch_output_b(const OutputArgs* args, const unsigned* start, int n, unsigned total,
                           hipStream_t s);
hipError_t launch_warm_b(const WarmArgs* args, const unsigned* start, int n, unsigned total,
                         hipStream_t s);
unsigned work_cg(const CgArgs& a, int C);
hipError_t launch_cg_dir_b(const CgArgs* args, const unsigned* start, int n, unsigned total,
                           hipStream_t s);
hipError_t launch_cg_step_b(const CgArgs* args, const unsigned* start, int n, unsigned total,
                            hipStream_t s);

// Launchers (all enqueue on `s`, return hipError_t of the launch).
// Stage f and mask into level 0 (b = C f, c, and u = C f when u != nullptr),
// check the input, and reduce ||b - A C f||^2 per channel into den.out.
hipError_t launch_stage(const float* f, const uint8_t* mask, int W, int H, int C, int Pf,
                        LevelView lv, uint8_t* c, float* b, float* u, int* status, NormOut den,
                        hipStream_t s);
// One pyramid level: coarse mask (max pool) and coarse known values
// (unscaled); the fine level is float32 when fine_f32.
hipError_t launch_rhs_down(LevelView fine, const uint8_t* cf, const void* bf, LevelView coarse,
                           uint8_t* cc, void* bc, int C, int naive, int prec, int fine_f32,
                           hipStream_t s);
hipError_t launch_pass(int mode, const PassArgs& a, int C, hipStream_t s);
hipError_t launch_restrict(const RestrictArgs& a, int C, hipStream_t s);
hipError_t launch_block_solve(const BlockArgs& a, int C, hipStream_t s);
hipError_t launch_coarse_solve(const CoarseArgs& a, int C, hipStream_t s);
hipError_t launch_output(LevelView lv, const uint8_t* c, const float* b,
                         const float* const* u_sel, float* out, int Pout, int C, hipStream_t s);
hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s);
// cgstat[ch][3] += (sum of itot, max of imax, sum of itot x block pixels) over
// the blocks of one level.
hipError_t launch_cg_stats(LevelView lv, const int* itot, const int* imax, int C,
                           unsigned long long* cgstat, hipStream_t s);

size_t pass_tiles(const LevelView& lv);
size_t prec_bytes(int prec);

}  // namespace inpaint
