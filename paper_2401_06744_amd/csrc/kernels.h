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

// One grid level as the kernels see it.  Fields are planar per channel with a
// padded row pitch P (elements); one plane holds H*P elements.
struct LevelView {
  int W, H, P;
  size_t plane;
  int nbx, nby;  // ORAS blocks along x and y
  int B, o;      // block side and overlap (stride B - o)
};

// Per-channel norm reduction of a grid pass.  Every workgroup publishes its
// partial sum and bumps a per-channel counter; the workgroup that arrives last
// adds all partials in a fixed order (see reduce_norm in kernels.hip).
struct NormOut {
  double* partials;   // [C][ntiles], every entry < 0 (unset) between passes
  unsigned* counter;  // [C][kCounterLines][32]: 64 group counters + 1 total, one
                      // 128-byte line each, all 0 between passes
  int* status;        // bit 2 (value 4) set if a partial never arrived
  double* out;        // [C] squared norm of the residual written by the pass
  // Optional convergence test on the finest grid (check != 0):
  const double* den;  // [C] squared norm of the reference residual
  double* relres;     // [C] sqrt(out / den)
  int* active;        // [C] set to 0 once relres <= tol
  double tol;
  int check;
};

enum PassMode : int {
  PASS_RES = 0,    // u_new = u_in (residual only; u_out unused)
  PASS_UPD = 1,    // u_new = u_in + sum of weighted block corrections
  PASS_PSOL = 2,   // u_new = mask ? b : P u_c   (cascade prolongation)
  PASS_PCORR = 3,  // u_new = u_in + (mask ? 0 : P u_c)   (coarse-grid correction)
};

struct PassArgs {
  LevelView lv;
  const uint8_t* c;
  const float* b;
  const float* u_in;
  float* u_out;
  float* r;
  const float* contrib;  // PASS_UPD: [C][nby*nbx][B][B]
  const float* uc;       // PASS_PSOL/PCORR: coarse field [C][Hc][Pc]
  int Wc, Hc, Pc;
  size_t planec;
  NormOut norm;
  const int* active;     // [C] or nullptr: skip channels already converged
  // PASS_UPD with rest != 0: instead of writing the fine residual and its norm,
  // restrict it (Sections 4.1, 4.4) to the coarse level: write bc = uc0 = rc's
  // right-hand side, uc0 = 0, rc = bc, and reduce the coarse norm into `norm`.
  int rest;
  LevelView clv;
  const uint8_t* cc;
  float* bc;
  float* uc0;
  float* rc;
};

struct BlockArgs {
  LevelView lv;
  const uint8_t* c;
  const float* r;         // residual [C][H][P]
  const double* snorm;    // [C] squared global residual norm
  float* contrib;         // [C][nby*nbx][B][B] weighted corrections D_i v_i
  float gamma, tau;
  int maxit;
  const int* active;
  int* itot;              // [C][nby*nbx] running total of local CG iterations per block,
  int* imax;              // and the running maximum; both nullptr to skip
};

struct CoarseArgs {
  LevelView lv;  // a single block covers the level
  const uint8_t* c;
  const float* b;
  float* u;      // in/out
  int init;      // 1: start from u = C b;  0: continue from u
  float rel_tol; // stop when ||rho||^2 <= rel_tol * ||rho_0||^2
  int maxit;
  const int* active;
};

// Launchers (all enqueue on `s`, return hipError_t of the launch).
// Stage f and mask into level 0 (b = C f, c, and u = C f when u != nullptr),
// check the input, and reduce ||b - A C f||^2 per channel into den.out.
hipError_t launch_stage(const float* f, const uint8_t* mask, int W, int H, int C, int Pf,
                        LevelView lv, uint8_t* c, float* b, float* u, int* status, NormOut den,
                        hipStream_t s);
hipError_t launch_mask_down(LevelView fine, const uint8_t* cf, LevelView coarse, uint8_t* cc,
                            hipStream_t s);
hipError_t launch_rhs_down(LevelView fine, const uint8_t* cf, const float* bf, LevelView coarse,
                           const uint8_t* cc, float* bc, int C, int naive, hipStream_t s);
hipError_t launch_pass(int mode, const PassArgs& a, int C, hipStream_t s);
hipError_t launch_restrict(LevelView fine, const float* rf, LevelView coarse, const uint8_t* cc,
                           float* bc, float* uc, float* rc, NormOut norm, const int* active,
                           int C, hipStream_t s);
hipError_t launch_block_solve(const BlockArgs& a, int C, hipStream_t s);
hipError_t launch_coarse_solve(const CoarseArgs& a, int C, hipStream_t s);
hipError_t launch_output(LevelView lv, const uint8_t* c, const float* b,
                         const float* const* u_sel, float* out, int Pout, int C, hipStream_t s);
hipError_t launch_copy_in(const float* src, int W, int H, int C, int Psrc, float* dst, LevelView lv,
                          hipStream_t s);

hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s);
// cgstat[ch][3] += (sum of itot, max of imax, sum of itot x block pixels) over
// the blocks of one level.
hipError_t launch_cg_stats(LevelView lv, const int* itot, const int* imax, int C,
                           unsigned long long* cgstat, hipStream_t s);

size_t pass_tiles(const LevelView& lv);

}  // namespace inpaint
