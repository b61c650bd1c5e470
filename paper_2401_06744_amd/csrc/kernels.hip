// gfx950 kernels of the homogeneous diffusion inpainting solver.
//
// Fields are planar per channel with a padded row pitch; the mask is uint8
// (1 = known).  The finest grid's iterate, known values and residual are
// float32; the weighted block corrections and every field of the coarser
// levels are float32, float16 or bfloat16 ("correction precision"), with all
// arithmetic in float32 (residuals in float64) and 16-bit fields stored scaled
// (see Sc in kernels.h).  Level l uses the integer 5-point stencil
// h_l^2 L (diagonal = number of in-image neighbours, -1 per neighbour), so the
// operator of every level is  A_l = C_l + (I - C_l) h_l^2 L_l  and coarse
// right-hand sides carry the factor (H/h)^2 = 4 (Sections 2.2 and 4.1).
//
// Kernels:
//   stage        b_0 = C f, mask normalised to 0/1, u_0 = C f, input checks
//   rhs_down     one pyramid level: coarse mask by max pooling and coarse
//                known values, naive or modified (Section 4.3)
//   pass<MODE>   one fused grid pass: form the new iterate on a 64x32 tile plus
//                a 1-pixel halo in LDS (ORAS update, cascade prolongation or
//                coarse-grid correction), write it, write the float64-evaluated
//                residual and reduce its squared norm per channel
//   block_solve  the ORAS local problems (Section 3, Algorithm 2, step 2): one
//                wavefront per block, the block held in registers, plain CG
//   restrict     coarse right-hand side of the correction problem (Section 4.1)
//   coarse_solve CG on the single block of the coarsest grid
//   output       out = mask ? f : u
#include "kernels.h"

#include <math.h>

#include <type_traits>

namespace inpaint {
namespace {

constexpr int kWave = 64;
constexpr int kPassThreads = 256;

using f16 = _Float16;
using bf16 = __bf16;

template <class T>
constexpr bool is_f32() {
  return std::is_same<T, float>::value;
}

// Global-memory pointers.  The field pointers arrive inside argument structs
// read from memory, so the compiler cannot tell them from LDS pointers and
// would use flat instructions: 64-bit address arithmetic per access, and a
// wait for LDS results that also waits for every outstanding HBM access.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// Whether channel ch still iterates (no flags: always).  Tested before the
// kernel's first loads: a converged channel's workgroups then cost a flag read
// and no field traffic (testing it late, to overlap the flag's round trip with
// those loads, was not faster on a live channel and made a stopped one cost
// about half a full pass).
__device__ __forceinline__ bool channel_active(const int* active, int ch) {
  return !active || glb(active)[ch] != 0;
}

__device__ __forceinline__ float scale_of(Sc s, const float* rho, int ch) {
  return s.rel ? s.f * rho[ch] : s.f;
}

// One channel of a field with element type T: load and store float values,
// undoing and applying the channel's scale for 16-bit types.
template <class T>
struct Fld {
  gptr<T> p;
  float s, inv;
  __device__ __forceinline__ Fld(const void* base, size_t chan_off, Sc sc, const float* rho, int ch) {
    p = base ? glb((T*)base + chan_off) : nullptr;  // optional fields may be absent
    if constexpr (is_f32<T>()) {
      s = inv = 1.0f;
    } else {
      s = scale_of(sc, rho, ch);
      inv = __builtin_amdgcn_rcpf(s);  // the 16-bit value is rounded anyway
    }
  }
  __device__ __forceinline__ float ld(int i) const {
    if constexpr (is_f32<T>())
      return p[i];
    else
      return (float)p[i] * s;
  }
  __device__ __forceinline__ void st(int i, float v) const {
    if constexpr (is_f32<T>())
      p[i] = v;
    else
      p[i] = (T)(v * inv);
  }
};

template <class T>
struct Tag {
  using type = T;
};

// Calls fn(Tag<level type>, Tag<correction type>) for a precision and level.
template <class Fn>
hipError_t with_types(int prec, int level0, Fn&& fn) {
  switch (prec) {
    case PREC_F32: return fn(Tag<float>{}, Tag<float>{});
    case PREC_F16: return level0 ? fn(Tag<float>{}, Tag<f16>{}) : fn(Tag<f16>{}, Tag<f16>{});
    case PREC_BF16: return level0 ? fn(Tag<float>{}, Tag<bf16>{}) : fn(Tag<bf16>{}, Tag<bf16>{});
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// cross-lane helpers
// ---------------------------------------------------------------------------

// DPP wave_shr:1 -- lane i receives lane i-1; lane 0 receives 0.
__device__ __forceinline__ float lane_from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x138, 0xf, 0xf, true));
}
// DPP wave_shl:1 -- lane i receives lane i+1; lane 63 receives 0.
__device__ __forceinline__ float lane_from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x130, 0xf, 0xf, true));
}
// DPP row_shr:1 / row_shl:1 -- inside each row of 16 lanes, lane i receives
// lane i-1 (i+1); the first (last) lane of a row receives 0.
__device__ __forceinline__ float row_from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x111, 0xf, 0xf, true));
}
__device__ __forceinline__ float row_from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x101, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float readlane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Smallest normal float32.  The CG coefficients use the hardware reciprocal,
// which flushes subnormal inputs (1/x becomes inf): a local CG stops once its
// squared residual norm or p.Ap leaves the normal range.
constexpr float kTiny = 1.17549435e-38f;

// Sum over the 64 lanes of a fully active wavefront, in a fixed order; the
// result is uniform.  quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror and
// row_mirror build 16-lane sums, then the four row sums are added.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Workgroups are handed to the 8 XCDs round robin.  Remap them so that each
// XCD works on runs of kXcdRun consecutive work items (tiles or blocks, which
// share halo and overlap reads in that XCD's L2), the runs dealt out to the
// XCDs in turn: every XCD then holds an even share of every part of the grid,
// and of every problem of a batch, whatever their costs.  (One contiguous
// eighth of the grid per XCD left an XCD with the slow problems of a batch,
// or with the last problems still iterating, and was slower on a single
// frame too; the last partial round keeps the hardware order.)
constexpr unsigned kXcdRun = 16;
__device__ __forceinline__ unsigned xcd_remap(unsigned wg, unsigned n) {
  const unsigned full = n - n % (8u * kXcdRun);
  if (wg >= full) return wg;
  const unsigned xcd = wg & 7u, idx = wg >> 3;  // the idx-th work item of this XCD
  return ((idx / kXcdRun) * 8u + xcd) * kXcdRun + idx % kXcdRun;
}

// Problem owning global work item g of a batched launch: the largest p with
// start[p] <= g (start[0] = 0, start[n] = total).
__device__ __forceinline__ int find_problem(const unsigned* __restrict__ start, int n, unsigned g) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__host__ __device__ __forceinline__ unsigned px_groups(int W, int H) {
  return (unsigned)((W + 63) / 64) * (unsigned)((H + 3) / 4);
}

// ---------------------------------------------------------------------------
// staging and output
// ---------------------------------------------------------------------------

// 64 x 16 pixels of one channel per workgroup, four rows per thread, loads
// issued together from clamped addresses.
constexpr int kOutRows = 4;
__device__ __forceinline__ void output_body(const OutputArgs& a, unsigned lin) {
  const LevelView& lv = a.lv;
  const unsigned gxn = (unsigned)((lv.W + 63) / 64);
  const unsigned per = gxn * (unsigned)((lv.H + 4 * kOutRows - 1) / (4 * kOutRows));
  const int ch = lin / per;
  const unsigned q = lin - (unsigned)ch * per;
  const int x = (int)(q % gxn) * 64 + (threadIdx.x & 63);
  const int y0 = (int)(q / gxn) * 4 * kOutRows + (threadIdx.x >> 6);
  if (x >= lv.W) return;
  // select without indexing the argument array dynamically (that would place
  // the arguments in scratch memory)
  const float* up = ch == 0 ? a.u[0] : ch == 1 ? a.u[1] : ch == 2 ? a.u[2] : a.u[3];
  if (a.flags) {
    const gptr<const int> blk = glb(a.flags);
    const int s0 = blk[12];
    int known = 0;
#pragma unroll
    for (int i = 0; i < kKnownWords; ++i) known |= blk[12 + kKnownAt + i];
    // a non-finite known value, no known pixel, or a lost norm partial: the
    // host reports the problem and nothing is written
    if ((s0 & 5) || !((s0 | known) & 2)) return;
    const double rr = ((const gptr<const double>)blk)[ch];
    if (blk[8 + ch] != 0 && isfinite(rr)) return;  // still iterating
    const int k = blk[16 + ch];
    if (k < 1 || k > a.nplan) return;
    const int cb = k == 1 ? a.cur[0] : (k - 2) % a.ncycle == 0 ? a.cur[1] : a.cur[2];
    up = cb == 0 ? a.u[0] : a.u[1];
  }
  const gptr<const float> u = glb(up);
  // ||b - A C f|| = 0: C f solves the channel exactly (0 at unknown pixels)
  const bool exact = a.den && a.den[ch] == 0.0;
  uint8_t k[kOutRows];
  float bv[kOutRows], uv[kOutRows];
#pragma unroll
  for (int r = 0; r < kOutRows; ++r) {
    const size_t o = (size_t)min(y0 + 4 * r, lv.H - 1) * lv.P + x;
    k[r] = glb(a.c)[o];
    bv[r] = glb(a.b)[(size_t)ch * lv.plane + o];
    uv[r] = u[(size_t)ch * lv.plane + o];
  }
#pragma unroll
  for (int r = 0; r < kOutRows; ++r) {
    const int y = y0 + 4 * r;
    if (y < lv.H)
      glb(a.out)[(size_t)ch * a.Pout * lv.H + (size_t)y * a.Pout + x] = k[r] ? bv[r] : (exact ? 0.0f : uv[r]);
  }
}

// The initial guess of a warm-started solve, laid out as the output (64
// columns x kOutRows rows every 4 per workgroup): u = known ? b : src, the
// caller's buffer read with its own pitch.
__device__ __forceinline__ void warm_body(const WarmArgs& a, unsigned lin) {
  const LevelView& lv = a.lv;
  const unsigned gxn = (unsigned)((lv.W + 63) / 64);
  const unsigned per = gxn * (unsigned)((lv.H + 4 * kOutRows - 1) / (4 * kOutRows));
  const int ch = lin / per;
  const unsigned q = lin - (unsigned)ch * per;
  const int x = (int)(q % gxn) * 64 + (threadIdx.x & 63);
  const int y0 = (int)(q / gxn) * 4 * kOutRows + (threadIdx.x >> 6);
  if (x >= lv.W) return;
  uint8_t k[kOutRows];
  float bv[kOutRows], sv[kOutRows];
#pragma unroll
  for (int r = 0; r < kOutRows; ++r) {
    const int y = min(y0 + 4 * r, lv.H - 1);
    const size_t o = (size_t)y * lv.P + x;
    k[r] = glb(a.c)[o];
    bv[r] = glb(a.b)[(size_t)ch * lv.plane + o];
    sv[r] = glb(a.src)[(size_t)ch * a.Psrc * lv.H + (size_t)y * a.Psrc + x];
  }
#pragma unroll
  for (int r = 0; r < kOutRows; ++r) {
    const int y = y0 + 4 * r;
    if (y < lv.H) glb(a.u)[(size_t)ch * lv.plane + (size_t)y * lv.P + x] = k[r] ? bv[r] : sv[r];
  }
}

// ---------------------------------------------------------------------------
// coarse problems (Section 4.3)
// ---------------------------------------------------------------------------

// One level of the coarse problems (Section 4.3) for a tile of 64 x 4 coarse
// cells: the coarse mask (max pool over the existing children; a child past
// the image edge repeats the existing one) and the coarse known value.
// Modified form: a known child j is weighted by its number of direct
// neighbours that are not known, judging a neighbour in the same cell by the
// fine mask and one in an adjacent cell by that cell's coarse mask (pooled
// here from the fine mask, so that both pyramids take one launch per level);
// neighbours outside the image are not counted.  If every weight is 0 the
// plain mean of the known children is used.  The fine mask of the tile's
// cells and their neighbours is staged in LDS, then the coarse masks of the
// tile's cells plus a one-cell ring; every cell is then worked out from LDS.
constexpr int kRhsCW = 64, kRhsCH = 4;  // coarse cells per workgroup (x, y)
template <class TF, class TC>
__device__ __forceinline__ void rhs_body(const RhsArgs& a, unsigned lin) {
  const LevelView& fl = a.fl;
  const LevelView& cl = a.cl;
  const gptr<const uint8_t> cf = glb(a.cf);
  const gptr<uint8_t> cc = glb(a.cc);
  const TF* __restrict__ bf = (const TF*)a.bf;
  TC* __restrict__ bc = (TC*)a.bc;
  const int C = a.C, naive = a.naive;
  const unsigned gxn = (unsigned)((cl.W + kRhsCW - 1) / kRhsCW);
  const int X0 = (int)(lin % gxn) * kRhsCW, Y0 = (int)(lin / gxn) * kRhsCH;
  // fine mask over columns 2 X0 - 2 .. 2 X0 + 2 kRhsCW + 1 and rows
  // 2 Y0 - 2 .. 2 Y0 + 2 kRhsCH + 1 (0 outside the image), and the coarse
  // masks of cells X0 - 1 .. X0 + kRhsCW, Y0 - 1 .. Y0 + kRhsCH
  constexpr int FW = 2 * kRhsCW + 4, FH = 2 * kRhsCH + 4, MW = kRhsCW + 2, MH = kRhsCH + 2;
  __shared__ uint8_t fm[FH][FW];
  __shared__ uint8_t pm[MH][MW];
  const int fx0 = 2 * X0 - 2, fy0 = 2 * Y0 - 2;
  for (int i = threadIdx.x; i < FH * FW; i += blockDim.x) {
    const int y = fy0 + i / FW, x = fx0 + i % FW;
    const bool in = y >= 0 && y < fl.H && x >= 0 && x < fl.W;
    fm[i / FW][i % FW] = in && cf[(size_t)(in ? y : 0) * fl.P + (in ? x : 0)] != 0;
  }
  __syncthreads();
  const auto fmask = [&](int y, int x) -> uint8_t { return fm[y - fy0][x - fx0]; };
  for (int i = threadIdx.x; i < MH * MW; i += blockDim.x) {
    const int cy = Y0 - 1 + i / MW, cx = X0 - 1 + i % MW;
    uint8_t m = 0;
    if (cx >= 0 && cy >= 0 && cx < cl.W && cy < cl.H) {
      const int xa = 2 * cx, ya = 2 * cy, xb = min(xa + 1, fl.W - 1), yb = min(ya + 1, fl.H - 1);
      m = ((fmask(ya, xa) | fmask(ya, xb)) | (fmask(yb, xa) | fmask(yb, xb))) ? 1 : 0;
    }
    pm[i / MW][i % MW] = m;
  }
  __syncthreads();
  const int X = X0 + (int)(threadIdx.x % kRhsCW), Y = Y0 + (int)(threadIdx.x / kRhsCW);
  if (X >= cl.W || Y >= cl.H) return;
  const size_t oc = (size_t)Y * cl.P + X;
  const uint8_t m = pm[Y - Y0 + 1][X - X0 + 1];
  cc[oc] = m;
  if (!m) {
    for (int ch = 0; ch < C; ++ch) bc[(size_t)ch * cl.plane + oc] = (TC)0.0f;
    return;
  }
  int wts[4];
  size_t offs[4];
  int nk = 0;
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      const int y = 2 * Y + dy, x = 2 * X + dx;
      if (y >= fl.H || x >= fl.W) continue;
      if (!fmask(y, x)) continue;
      int w = 0;
      const int ny[4] = {y, y, y - 1, y + 1};
      const int nx[4] = {x - 1, x + 1, x, x};
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int yy = ny[d], xx = nx[d];
        if (yy < 0 || yy >= fl.H || xx < 0 || xx >= fl.W) continue;
        const bool same = (yy >> 1) == Y && (xx >> 1) == X;
        const uint8_t k = same ? fmask(yy, xx) : pm[(yy >> 1) - Y0 + 1][(xx >> 1) - X0 + 1];
        w += k ? 0 : 1;
      }
      wts[nk] = w;
      offs[nk] = (size_t)y * fl.P + x;
      ++nk;
    }
  int wsum = 0;
  for (int k = 0; k < nk; ++k) wsum += wts[k];
  for (int ch = 0; ch < C; ++ch) {
    const TF* bp = bf + (size_t)ch * fl.plane;
    double num = 0.0, plain = 0.0;
    for (int k = 0; k < nk; ++k) {
      const double v = (double)(float)bp[offs[k]];
      num += (double)wts[k] * v;
      plain += v;
    }
    double val;
    if (!naive && wsum > 0)
      val = num / (double)wsum;
    else
      val = plain / (double)(nk > 0 ? nk : 1);
    bc[(size_t)ch * cl.plane + oc] = (TC)(float)val;
  }
}

// ---------------------------------------------------------------------------
// norm reduction inside the pass: the last workgroup adds the partials
// ---------------------------------------------------------------------------
//
// On gfx950 the L2 caches of the eight XCDs are not coherent with each other
// and a device-scope release fence writes back the whole L2.  Instead, each
// workgroup writes its partial with an agent-scope atomic store (written
// through to the coherent level) and then increments a per-channel counter
// with an agent-scope atomic.  The workgroup that sees the count reach
// ntiles - 1 reads the partials with agent-scope atomic loads; an entry is
// "unset" while it holds the kUnsetPartialBits pattern (a NaN payload that no
// arithmetic produces; partials may be negative), so it waits for the few that
// may still be in flight, adds them in index order (a result that does not
// depend on which workgroup came last), resets every entry to the pattern and
// the counter to 0 for the next pass, and runs the optional convergence test.
constexpr int kSpinBudget = 1 << 20;

__device__ __forceinline__ bool unset(double v) {
  return (unsigned long long)__builtin_bit_cast(long long, v) == kUnsetPartialBits;
}

__device__ void reduce_norm(double acc, int ch, unsigned tile, unsigned ntiles, const NormOut& no) {
  constexpr int NW = kPassThreads / kWave;
  __shared__ double red[NW];
  __shared__ int last;
  if (no.mode == NORM_NONE) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  acc = wave_sum_d(acc);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (no.mode == NORM_DEFER) {
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += red[w];
      no.dpart[(size_t)ch * no.dstride + tile] = s;
    }
    return;
  }
  double* part = no.partials + (size_t)ch * ntiles;
  unsigned* cnt = no.counter + (size_t)ch * kCounterLines * 32;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w];
    __hip_atomic_store(part + tile, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // two-level count: tile -> group (tile mod 64) -> total, so that no
    // counter sees more than ~ntiles/64 increments
    const unsigned grp = tile % kCounterGroups;
    const unsigned ngrp = ntiles < (unsigned)kCounterGroups ? ntiles : (unsigned)kCounterGroups;
    const unsigned gsize = (ntiles - grp + kCounterGroups - 1) / kCounterGroups;
    const unsigned prev =
        __hip_atomic_fetch_add(cnt + grp * 32, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int l = 0;
    if (prev == gsize - 1) {
      const unsigned tp = __hip_atomic_fetch_add(cnt + kCounterGroups * 32, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
      l = tp == ngrp - 1;
    }
    last = l;
  }
  __syncthreads();
  if (!last) return;
  // Entries t, t + T, t + 2T, ... are added in that order; loads are issued in
  // batches of U so that the coherent-level round trips overlap.
  constexpr int U = 8;
  double s = 0.0;
  int spins = 0;
  bool lost = false;
  for (unsigned base = threadIdx.x; base < ntiles; base += U * kPassThreads) {
    double v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const unsigned i = base + j * kPassThreads;
      v[j] = i < ntiles ? __hip_atomic_load(part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const unsigned i = base + j * kPassThreads;
      if (i >= ntiles) continue;
      while (unset(v[j]) && spins < kSpinBudget) {
        __builtin_amdgcn_s_sleep(1);
        ++spins;
        v[j] = __hip_atomic_load(part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (unset(v[j])) {
        lost = true;
        v[j] = 0.0;
      }
      s += v[j];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const unsigned i = base + j * kPassThreads;
      if (i < ntiles)
        __hip_atomic_store(part + i, __builtin_bit_cast(double, kUnsetPartialBits), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  s = wave_sum_d(s);
  __syncthreads();
  if (lane == 0) red[wave] = s;
  if (lost) atomicOr(no.status, 4);
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < NW; ++w) tot += red[w];
    no.out[ch] = tot;
    if (no.rho) no.rho[ch] = (float)fmax(sqrt(tot * no.inv_n), 1e-30);
    for (int gi = 0; gi < kCounterLines; ++gi)
      __hip_atomic_store(cnt + gi * 32, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (no.check) {
      const double den = no.den[ch];
      // den = 0: A C f = b, so C f is the exact solution; the output writes
      // it, and the channel counts as converged at its first test
      const double rel = den > 0.0 ? sqrt(tot / den) : 0.0;
      no.relres[ch] = rel;
      // converged, or diverged (a non-finite residual): the channel stops
      if (rel <= no.tol || !(rel < INFINITY)) no.active[ch] = 0;
      if (no.checks) no.checks[ch] += 1;
    }
  }
}

// Local CG statistics of one level: one workgroup per channel.
__global__ void __launch_bounds__(kPassThreads) k_cg_stats(LevelView lv, const int* __restrict__ itot,
                                                          const int* __restrict__ imax,
                                                          unsigned long long* __restrict__ cgstat) {
  constexpr int NW = kPassThreads / kWave;
  __shared__ unsigned long long red[3][NW];
  const int ch = blockIdx.x;
  const unsigned nblk = (unsigned)(lv.nbx * lv.nby);
  const int S = lv.B - lv.o;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long isum = 0, mx = 0, ipx = 0;
  for (unsigned i = threadIdx.x; i < nblk; i += kPassThreads) {
    const unsigned long long it = (unsigned)itot[(size_t)ch * nblk + i];
    const unsigned long long im = (unsigned)imax[(size_t)ch * nblk + i];
    const int bx = (int)(i % (unsigned)lv.nbx), by = (int)(i / (unsigned)lv.nbx);
    const int bw = min(lv.B, lv.W - bx * S), bh = min(lv.B, lv.H - by * S);
    isum += it;
    mx = im > mx ? im : mx;
    ipx += it * (unsigned long long)(bw * bh);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    isum += __shfl_xor(isum, m);
    const unsigned long long om = __shfl_xor(mx, m);
    mx = om > mx ? om : mx;
    ipx += __shfl_xor(ipx, m);
  }
  if (lane == 0) {
    red[0][wave] = isum;
    red[1][wave] = mx;
    red[2][wave] = ipx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long* cs = cgstat + 3 * ch;
    for (int w = 0; w < NW; ++w) {
      cs[0] += red[0][w];
      cs[1] = red[1][w] > cs[1] ? red[1][w] : cs[1];
      cs[2] += red[2][w];
    }
  }
}

// Sets every norm partial to the unset pattern once per workspace.
__global__ void k_fill(double* p, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// staging of the finest level
// ---------------------------------------------------------------------------

// One 64x32 tile of one channel: b = C f, c and (optionally) u = C f for the
// tile, input checks, and the residual of C f (the reference residual of the
// relative residual):  at an unknown pixel it is the sum of the known
// neighbours' values, at a known pixel 0.
__device__ __forceinline__ void stage_body(const StageArgs& a, unsigned lin) {
  const gptr<const float> f = glb(a.f);
  const gptr<const uint8_t> mask = glb(a.mask);
  const int W = a.W, H = a.H, Pf = a.Pf;
  const LevelView& lv = a.lv;
  const gptr<uint8_t> c = glb(a.c);
  const gptr<float> b = glb(a.b);
  const gptr<float> u = a.u ? glb(a.u) : nullptr;
  int* __restrict__ status = a.status;
  const NormOut& den = a.den;
  const unsigned tiles_x = (unsigned)((lv.W + kTileW - 1) / kTileW);
  const unsigned ntiles = tiles_x * (unsigned)((lv.H + kTileH - 1) / kTileH);
  const int ch = lin / ntiles;
  const unsigned tile = lin - (unsigned)ch * ntiles;
  const int x0 = (int)(tile % tiles_x) * kTileW, y0 = (int)(tile / tiles_x) * kTileH;
  __shared__ float t[kTileH + 2][kTileW + 2];
  __shared__ uint8_t kn[kTileH + 2][kTileW + 2];
  const gptr<const float> fc = f + (size_t)ch * Pf * H;
  bool bad = false, any = false;
  // Phase 1, laid out as the grid passes: thread (column c, row group g)
  // takes column x0 + c of tile rows g, g + 4, ... (the tile plus a one-pixel
  // halo row above and below; rows past the halo repeat a valid row and are
  // not kept); a few threads take the two halo columns.  Mask and f are read
  // from clamped in-image addresses up front (f at unknown pixels is read but
  // never used); pixels outside the image enter the tile as unknown, 0.
  constexpr int TW = kTileW + 2, TH = kTileH + 2;
  constexpr int NG = kPassThreads / kTileW;
  constexpr int RJ = (TH + NG - 1) / NG;
  const int cc = threadIdx.x & (kTileW - 1), g = threadIdx.x / kTileW;
  const int gx = x0 + cc;
  const int gxc = min(gx, W - 1);
  uint8_t km[RJ];
  float fv[RJ];
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int ty = min(g + NG * j, TH - 1);
    const int gy = min(max(y0 - 1 + ty, 0), H - 1);
    km[j] = mask[(size_t)gy * W + gxc];
    fv[j] = fc[(size_t)gy * Pf + gxc];
  }
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int ty = g + NG * j;
    if (ty >= TH) break;
    const int gy = y0 - 1 + ty;
    const bool in = gx < W && gy >= 0 && gy < H;
    const uint8_t k = in && km[j] != 0;
    const float v = k ? fv[j] : 0.0f;
    if (in && ty >= 1 && ty <= kTileH) {
      bad |= k && !isfinite(v);
      any |= k;
      const size_t oc = (size_t)gy * lv.P + gx;
      if (ch == 0) c[oc] = k;
      b[(size_t)ch * lv.plane + oc] = v;
      if (u) u[(size_t)ch * lv.plane + oc] = v;
    }
    t[ty][cc + 1] = v;
    kn[ty][cc + 1] = k;
  }
  if (threadIdx.x < 2 * TH) {
    // halo columns tx = 0 and tx = TW - 1 (kept in LDS only)
    const int side = threadIdx.x / TH, ty = threadIdx.x - side * TH;
    const int hx = side == 0 ? x0 - 1 : x0 + kTileW, hy = y0 - 1 + ty;
    const int hxc = min(max(hx, 0), W - 1), hyc = min(max(hy, 0), H - 1);
    const uint8_t hm = mask[(size_t)hyc * W + hxc];
    const float hf = fc[(size_t)hyc * Pf + hxc];
    const uint8_t k = hx >= 0 && hx < W && hy >= 0 && hy < H && hm != 0;
    t[ty][side == 0 ? 0 : TW - 1] = k ? hf : 0.0f;
    kn[ty][side == 0 ? 0 : TW - 1] = k;
  }
  // Report: a non-finite known value (rare) by an atomic OR into status[0];
  // "a known pixel exists" (nearly every tile) by a plain store of 2 into the
  // known word of this workgroup's XCD, which only that XCD's workgroups write
  // (the same value: no read-modify-write, nothing to wait for, and no
  // address that every workgroup of the launch contends for).
  const unsigned long long anybad = __ballot(bad);
  const unsigned long long anyknown = __ballot(any);
  if ((threadIdx.x & 63) == 0) {
    if (anybad) atomicOr(status, 1);
    if (anyknown) status[kKnownAt + (blockIdx.x & (kKnownWords - 1))] = 2;
  }
  __syncthreads();
  const int tx = cc, tyg = g;  // phase 2: 8 rows of column gx per thread
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kTileH / 4; ++k) {
    const int ty = tyg * (kTileH / 4) + k;
    const int gy = y0 + ty;
    if (gx < W && gy < H && !kn[ty + 1][tx + 1]) {
      double nsum = 0.0;
      if (gx > 0) nsum += (double)t[ty + 1][tx];
      if (gx < W - 1) nsum += (double)t[ty + 1][tx + 2];
      if (gy > 0) nsum += (double)t[ty][tx + 1];
      if (gy < H - 1) nsum += (double)t[ty + 2][tx + 1];
      acc += nsum * nsum;
    }
  }
  reduce_norm(acc, ch, tile, ntiles, den);
}

// ---------------------------------------------------------------------------
// fused grid pass
// ---------------------------------------------------------------------------

// Floor division by a small positive divisor that is the same for the whole
// grid, through a float reciprocal and one correction step (exact for n < 2^24).
__device__ __forceinline__ int div_small(int n, int d, float rd) {
  int q = (int)((float)n * rd);
  q += (q + 1) * d <= n ? 1 : 0;
  q -= q * d > n ? 1 : 0;
  return q;
}

// Where pixel index g (along one axis) sits in the ORAS blocks: the block b1
// whose start is the last at or before g, the local index l1 in it, whether the
// previous block also covers g (h0), and the parts of the correction-buffer
// offset for this axis.
struct BlockAxis {
  int b1, l1;
  bool h0;
};
__device__ __forceinline__ BlockAxis block_axis(int g, int S, float rS, int o, int nb) {
  BlockAxis r;
  r.b1 = min(div_small(g, S, rS), nb - 1);
  r.l1 = g - r.b1 * S;
  r.h0 = r.b1 > 0 && r.l1 < o;
  return r;
}

// Bilinear cell-centred prolongation weights along one axis: fine index g maps
// to the nearest coarse index n and the second one f (clamped at the edge).
__device__ __forceinline__ void prolong_axis(int g, int nc, int& n, int& f) {
  n = g >> 1;
  f = (g & 1) ? min(n + 1, nc - 1) : max(n - 1, 0);
}

__device__ __forceinline__ double bilinear(double a, double b, double c, double d) {
  // ((9/16 a + 3/16 b) + 3/16 c) + 1/16 d, each product and sum rounded once
  double s = __dadd_rn(__dmul_rn(0.5625, a), __dmul_rn(0.1875, b));
  s = __dadd_rn(s, __dmul_rn(0.1875, c));
  return __dadd_rn(s, __dmul_rn(0.0625, d));
}

// what a pass mode reads and writes
__host__ __device__ constexpr bool mode_upd(int m) {
  return m == PASS_UPD || m == PASS_UPD0 || m == PASS_FIN || m == PASS_FIN0;
}
__host__ __device__ constexpr bool mode_contrib(int m) {
  return m == PASS_UPD || m == PASS_UPD0 || m == PASS_FIN;
}
__host__ __device__ constexpr bool mode_pcorr(int m) { return m == PASS_PCORR || m == PASS_PCORR0; }
__host__ __device__ constexpr bool mode_zero(int m) { return m == PASS_UPD0 || m == PASS_PCORR0; }
__host__ __device__ constexpr bool mode_fin(int m) { return m == PASS_FIN || m == PASS_FIN0; }
__host__ __device__ constexpr bool mode_rest(int m) { return m == PASS_UPD || m == PASS_UPD0; }

// Coarse patch of a 64 x 32 tile's prolongation: the tile and its 1-pixel halo
// span at most 34 coarse columns and 18 coarse rows.
constexpr int kCoarseW = kTileW / 2 + 2, kCoarseH = kTileH / 2 + 2;

// Two horizontally adjacent pixels (an even column and the next one).
struct Px2 {
  float v[2];
};

// Pair loads and stores of a field: element i must be even (i.e. the pair is
// 2-element aligned); one 8-byte (float32) or 4-byte (16-bit) access.
template <class T>
__device__ __forceinline__ Px2 ld2(const Fld<T>& f, int i) {
  Px2 r;
  if constexpr (is_f32<T>()) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(const __attribute__((address_space(1))) v2*)(f.p + i);
    r.v[0] = v.x;
    r.v[1] = v.y;
  } else {
    const unsigned w = *(const __attribute__((address_space(1))) unsigned*)(f.p + i);
    const T lo = __builtin_bit_cast(T, (unsigned short)(w & 0xffffu));
    const T hi = __builtin_bit_cast(T, (unsigned short)(w >> 16));
    r.v[0] = (float)lo * f.s;
    r.v[1] = (float)hi * f.s;
  }
  return r;
}
template <class T>
__device__ __forceinline__ void st2(const Fld<T>& f, int i, float a, float b) {
  if constexpr (is_f32<T>()) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    *(__attribute__((address_space(1))) v2*)(f.p + i) = v2{a, b};
  } else {
    const T ta = (T)(a * f.inv), tb = (T)(b * f.inv);
    *(__attribute__((address_space(1))) unsigned*)(f.p + i) =
        (unsigned)__builtin_bit_cast(unsigned short, ta) | ((unsigned)__builtin_bit_cast(unsigned short, tb) << 16);
  }
}
// Known flags of the pixel pair at an even offset.
__device__ __forceinline__ unsigned short ld_mask2(const uint8_t* c, int i) {
  return *(const __attribute__((address_space(1))) unsigned short*)(c + i);
}

// New iterate of a pixel (or of an aligned pixel pair) for one pass mode.
// Column data is computed once per thread, row data per row.  TU: element
// type of this level's iterate and known values; TC: corrections and the
// coarse field.  The pair functions rely on an even block stride and overlap:
// both pixels of an aligned pair then lie in the same blocks at the same
// overlap side, so that their four weighted corrections are four pair loads.
template <int MODE, class TU, class TC>
struct Former {
  const PassArgs& a;
  Fld<TU> uin, bb;
  Fld<TC> cb, uc;   // corrections of this channel (UPD); coarse field (PSOL, PCORR)
  Fld<TC> ea;       // added correction (UPD with e_add)
  int S, o, B, nbx, nby;
  float rS;
  // PSOL/PCORR: the coarse cells the tile's bilinear stencils touch, staged
  // in LDS ([kCoarseH][kCoarseW] from coarse (cx0, cy0))
  const float* cpatch = nullptr;
  int cx0 = 0, cy0 = 0;

  __device__ Former(const PassArgs& a_, int ch)
      : a(a_),
        uin(a_.u_in, (size_t)ch * a_.lv.plane, a_.s_u, a_.rho, ch),
        bb(a_.b, (size_t)ch * a_.lv.plane, a_.s_b, a_.rho, ch),
        cb(a_.contrib, (size_t)ch * ((size_t)a_.lv.nbx * a_.lv.nby * a_.lv.B * a_.lv.B), a_.s_contrib,
           a_.rho, ch),
        uc(a_.uc, (size_t)ch * a_.planec, a_.s_uc, a_.rho, ch),
        ea(a_.e_add, (size_t)ch * a_.lv.plane, a_.s_e, a_.rho, ch) {
    const LevelView& lv = a.lv;
    B = lv.B;
    S = lv.B - lv.o;
    o = lv.o;
    nbx = lv.nbx;
    nby = lv.nby;
    rS = 1.0f / (float)S;
  }

  struct Col {
    int gx;
    int cx1, cx0;  // UPD: column part of the correction offsets of blocks bx1, bx1 - 1
    bool h0;
    int xn, xf;    // PSOL/PCORR: coarse columns (of the pair's first pixel)
  };
  __device__ Col col(int gx) const {
    Col c;
    c.gx = gx;
    if constexpr (mode_contrib(MODE)) {
      const BlockAxis ax = block_axis(gx, S, rS, o, nbx);
      c.cx1 = ax.b1 * B * B + ax.l1;
      c.cx0 = (ax.b1 - 1) * B * B + ax.l1 + S;
      c.h0 = ax.h0;
    }
    if constexpr (MODE == PASS_PSOL || mode_pcorr(MODE)) prolong_axis(gx, a.Wc, c.xn, c.xf);
    return c;
  }

  // Row offsets of the (up to) four blocks covering row gy: ry1 (block by1) and
  // ry0 (block by1 - 1, or ry1 when absent); h0y: the upper block is present.
  __device__ void rows(int gy, int& ry0, int& ry1, bool& h0y) const {
    const BlockAxis ay = block_axis(gy, S, rS, o, nby);
    ry1 = ay.b1 * nbx * B * B + ay.l1 * B;
    ry0 = ay.h0 ? (ay.b1 - 1) * nbx * B * B + (ay.l1 + S) * B : ry1;
    h0y = ay.h0;
  }

  // the same additions, in the same order, as adding only the present corrections
  static __device__ __forceinline__ float sum4(float d00, float d01, float d10, float d11, bool hy, bool hx) {
    return (((hy && hx ? d00 : 0.0f) + (hy ? d01 : 0.0f)) + (hx ? d10 : 0.0f)) + d11;
  }

  // single pixel (the halo columns)
  __device__ float value(const Col& c, int gy) const {
    const LevelView& lv = a.lv;
    const int off = gy * lv.P + c.gx;
    if constexpr (MODE == PASS_RES) {
      return uin.ld(off);
    } else if constexpr (mode_upd(MODE)) {
      float d = 0.0f;
      if constexpr (mode_contrib(MODE)) {
        // the upper blocks' slots only in the rows they cover (a branch that
        // is uniform over a wavefront but at the edges of those rows); the
        // left block's slot is read in every column, an absent one at a valid
        // stand-in address and then dropped (a branch per column, taken by
        // some lanes of every wavefront, saves nothing)
        int ry0, ry1;
        bool hy;
        rows(gy, ry0, ry1, hy);
        const int cx0 = c.h0 ? c.cx0 : c.cx1;
        float d00 = 0.0f, d01 = 0.0f;
        if (hy) {
          d00 = cb.ld(ry0 + cx0);
          d01 = cb.ld(ry0 + c.cx1);
        }
        const float d10 = cb.ld(ry1 + cx0), d11 = cb.ld(ry1 + c.cx1);
        d = sum4(d00, d01, d10, d11, hy, c.h0);
      }
      if constexpr (mode_fin(MODE)) d = ea.ld(off) + d;
      if constexpr (mode_zero(MODE))
        return d;
      else
        return uin.ld(off) + d;
    } else {
      const bool known = glb(a.c)[off] != 0;
      const float x = MODE == PASS_PSOL ? bb.ld(off) : (mode_zero(MODE) ? 0.0f : uin.ld(off));
      int yn, yf;
      prolong_axis(gy, a.Hc, yn, yf);
      return fin1(c.xn, c.xf, yn, yf, known, x);
    }
  }

  // the aligned pair at column c.gx (even): UPD and RES modes
  __device__ Px2 value2(const Col& c, int gy) const {
    const LevelView& lv = a.lv;
    const int off = gy * lv.P + c.gx;
    if constexpr (MODE == PASS_RES) {
      return ld2(uin, off);
    } else {
      Px2 d{{0.0f, 0.0f}};
      if constexpr (mode_contrib(MODE)) {
        int ry0, ry1;
        bool hy;
        rows(gy, ry0, ry1, hy);
        const int cx0 = c.h0 ? c.cx0 : c.cx1;
        Px2 d00{{0.0f, 0.0f}}, d01{{0.0f, 0.0f}};
        if (hy) {  // as in value()
          d00 = ld2(cb, ry0 + cx0);
          d01 = ld2(cb, ry0 + c.cx1);
        }
        const Px2 d10 = ld2(cb, ry1 + cx0), d11 = ld2(cb, ry1 + c.cx1);
#pragma unroll
        for (int h = 0; h < 2; ++h) d.v[h] = sum4(d00.v[h], d01.v[h], d10.v[h], d11.v[h], hy, c.h0);
      }
      if constexpr (mode_fin(MODE)) {
        const Px2 e = ld2(ea, off);
#pragma unroll
        for (int h = 0; h < 2; ++h) d.v[h] = e.v[h] + d.v[h];
      }
      if constexpr (!mode_zero(MODE)) {
        const Px2 u = ld2(uin, off);
#pragma unroll
        for (int h = 0; h < 2; ++h) d.v[h] = u.v[h] + d.v[h];
      }
      return d;
    }
  }

  // Prolongations in two steps: the pair's global inputs (known flags, and
  // the known values (PSOL) or iterate (PCORR)), then the values from the
  // coarse patch in LDS.
  struct Pre2 {
    unsigned short known;  // byte h: known flag of pixel h
    Px2 x;
  };
  __device__ Pre2 pre2(const Col& c, int gy) const {
    const int off = gy * a.lv.P + c.gx;
    Pre2 p;
    p.known = ld_mask2(a.c, off);
    if constexpr (MODE == PASS_PSOL)
      p.x = ld2(bb, off);  // read unconditionally: no branch around the load
    else if constexpr (mode_zero(MODE))
      p.x = Px2{{0.0f, 0.0f}};
    else
      p.x = ld2(uin, off);
    return p;
  }
  __device__ float fin1(int xn, int xf, int yn, int yf, bool known, float x) const {
    const float* rn = cpatch + (yn - cy0) * kCoarseW - cx0;
    const float* rf = cpatch + (yf - cy0) * kCoarseW - cx0;
    const double p = bilinear(rn[xn], rn[xf], rf[xn], rf[xf]);
    if constexpr (MODE == PASS_PSOL)
      return known ? x : (float)p;
    else
      return known ? x : (float)((double)x + p);
  }
  __device__ Px2 fin2(const Col& c, int gy, const Pre2& pr) const {
    int yn, yf;
    prolong_axis(gy, a.Hc, yn, yf);
    // the pair's first pixel is even: its second coarse column lies to the
    // left, the odd pixel's to the right (both clamped at the edge)
    const int xf1 = min(c.xn + 1, a.Wc - 1);
    Px2 r;
    r.v[0] = fin1(c.xn, c.xf, yn, yf, (pr.known & 0xffu) != 0, pr.x.v[0]);
    r.v[1] = fin1(c.xn, xf1, yn, yf, (pr.known >> 8) != 0, pr.x.v[1]);
    return r;
  }
};

// Coarse value (X, Y) read by a prolongation whose coarse level's last ORAS
// update was left to it: u + the (up to four) weighted block corrections of
// the coarse level, added in the order of the update pass, and rounded to the
// coarse field's type and scale as that pass would have stored it.
template <class TC>
__device__ __forceinline__ float coarse_updated(const PassArgs& a, const Fld<TC>& uc, int ch, int X, int Y) {
  const LevelView& cl = a.clv;
  const int B = cl.B, o = cl.o, S = B - o;
  const float rS = 1.0f / (float)S;
  const Fld<TC> cb(a.ccontrib, (size_t)ch * ((size_t)cl.nbx * cl.nby * B * B), a.s_contrib, a.rho, ch);
  const BlockAxis ax = block_axis(X, S, rS, o, cl.nbx);
  const BlockAxis ay = block_axis(Y, S, rS, o, cl.nby);
  const int cx1 = ax.b1 * B * B + ax.l1;
  const int cx0 = ax.h0 ? (ax.b1 - 1) * B * B + ax.l1 + S : cx1;
  const int ry1 = ay.b1 * cl.nbx * B * B + ay.l1 * B;
  const int ry0 = ay.h0 ? (ay.b1 - 1) * cl.nbx * B * B + (ay.l1 + S) * B : ry1;
  float d00 = 0.0f, d01 = 0.0f;
  if (ay.h0) {  // the upper blocks' slots only in the rows they cover
    d00 = cb.ld(ry0 + cx0);
    d01 = cb.ld(ry0 + cx1);
  }
  const float d10 = cb.ld(ry1 + cx0), d11 = cb.ld(ry1 + cx1);
  const float d = (((ay.h0 && ax.h0 ? d00 : 0.0f) + (ay.h0 ? d01 : 0.0f)) + (ax.h0 ? d10 : 0.0f)) + d11;
  const float un = uc.ld(Y * a.Pc + X) + d;
  if constexpr (is_f32<TC>())
    return un;
  else
    return (float)(TC)(un * uc.inv) * uc.s;
}

// One fused grid pass over a 64x32 tile of one channel.  Thread (pair column
// q, row group g) works on columns x0 + 2q and x0 + 2q + 1: every field access
// is a pair access.
//   phase 1: the new iterate on the tile plus a 1-pixel halo, into LDS.  A halo
//            pixel outside the image takes the value of the pixel it mirrors,
//            so that the reflecting boundary needs no special case below.
//   phase 2: write the iterate; residual r = b - u at known pixels and
//            r = b - (4u - (l + r + up + down)) elsewhere, in float64; write it
//            (or keep it in LDS for the fused restriction); norm partial.
template <int MODE, class TU, class TC>
__device__ __forceinline__ void pass_body(const PassArgs& a, unsigned lin) {
  constexpr int QW = kTileW / 2;             // pair columns per tile
  constexpr int NG = kPassThreads / QW;      // row groups
  constexpr int TH = kTileH + 2;
  // LDS row: halo column at index 1, tile column x at x + 2, halo at kTileW + 2
  // (pairs start at even indices)
  constexpr int TW = kTileW + 4;
  constexpr int RJ = (TH + NG - 1) / NG;     // phase-1 rows per thread
  constexpr int RK = kTileH / NG;            // phase-2 rows per thread
  static_assert(RJ == RK + 1 && kTileH == NG * RK, "row slots: RK tile rows and one halo slot");
  const unsigned tiles_x = (unsigned)((a.lv.W + kTileW - 1) / kTileW);
  const unsigned ntiles = tiles_x * (unsigned)((a.lv.H + kTileH - 1) / kTileH);
  const int ch = lin / ntiles;
  const unsigned tile = lin - (unsigned)ch * ntiles;
  if (!channel_active(a.active, ch)) return;  // the whole workgroup: one channel
  const LevelView& lv = a.lv;
  const int W = lv.W, H = lv.H;
  const int x0 = (int)(tile % tiles_x) * kTileW, y0 = (int)(tile / tiles_x) * kTileH;
  constexpr bool kProlong = MODE == PASS_PSOL || mode_pcorr(MODE);
  __shared__ float t[TH][TW];
  __shared__ float cp[kProlong ? kCoarseH : 1][kProlong ? kCoarseW : 1];
  Former<MODE, TU, TC> F(a, ch);
  const int q = threadIdx.x % QW, g = threadIdx.x / QW;
  const int gx = x0 + 2 * q;
  // the pair that is read: this thread's, or for columns past the image the
  // last in-image pair (its pixel W - 1 is the mirror of column W)
  const int gxe = min(gx, (W - 1) & ~1);
  const bool lastodd = ((W - 1) & 1) != 0;  // column W - 1 is the pair's second pixel
  // Rows: slot k < RK of thread row group g holds tile row g + NG k (LDS row
  // g + NG k + 1) in both phases, so that a prolongation's known flags of
  // phase 1 serve phase 2; slot RK holds the top halo row (g = 0) or the
  // bottom one (g = 1), and is idle for the other row groups.
  const auto slot_ty = [&](int j) { return j < RK ? g + NG * j + 1 : (g == 0 ? 0 : TH - 1); };
  const auto slot_on = [&](int j) { return j < RK || g < 2; };
  // Phase-2 inputs that do not depend on phase 1 (masks and right-hand sides
  // of this thread's rows) are loaded first, from clamped addresses, so that
  // their latency overlaps phase 1's.  (The final pass of the correction form
  // holds more phase-1 state and loads them for phase 2 instead.)
  unsigned short mk[RK];
  Px2 bvv[RK];
  if constexpr (!mode_fin(MODE)) {
    if constexpr (!kProlong) {  // a prolongation takes them from phase 1
#pragma unroll
      for (int k = 0; k < RK; ++k) mk[k] = ld_mask2(a.c, min(y0 + g + NG * k, H - 1) * lv.P + gxe);
    }
    if (MODE == PASS_RES || !a.solution) {
#pragma unroll
      for (int k = 0; k < RK; ++k) bvv[k] = ld2(F.bb, min(y0 + g + NG * k, H - 1) * lv.P + gxe);
    } else {
#pragma unroll
      for (int k = 0; k < RK; ++k) bvv[k] = Px2{{0.0f, 0.0f}};
    }
  }
  {
    const auto col = F.col(gxe);
    Px2 v[RJ];
    if constexpr (kProlong) {
      // the rows' own inputs first, then the coarse patch
      typename Former<MODE, TU, TC>::Pre2 pr[RJ];
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        if (!slot_on(j)) continue;
        pr[j] = F.pre2(col, min(max(y0 - 1 + slot_ty(j), 0), H - 1));
      }
      if constexpr (!mode_fin(MODE)) {
#pragma unroll
        for (int k = 0; k < RK; ++k) mk[k] = pr[k].known;
      }
      // coarse cells (x0/2 - 1 .. x0/2 + 32) x (y0/2 - 1 .. y0/2 + 16), clamped
      const int cx0 = max((x0 >> 1) - 1, 0), cy0 = max((y0 >> 1) - 1, 0);
      for (int i = threadIdx.x; i < kCoarseW * kCoarseH; i += kPassThreads) {
        const int py = i / kCoarseW, px = i - py * kCoarseW;
        const int X = min(cx0 + px, a.Wc - 1), Y = min(cy0 + py, a.Hc - 1);
        cp[py][px] = a.ccontrib ? coarse_updated<TC>(a, F.uc, ch, X, Y) : F.uc.ld(Y * a.Pc + X);
      }
      F.cpatch = &cp[0][0];
      F.cx0 = cx0;
      F.cy0 = cy0;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        if (!slot_on(j)) continue;
        v[j] = F.fin2(col, min(max(y0 - 1 + slot_ty(j), 0), H - 1), pr[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        if (!slot_on(j)) continue;  // the halo slot: wavefronts of row groups >= 2 skip it
        v[j] = F.value2(col, min(max(y0 - 1 + slot_ty(j), 0), H - 1));
      }
    }
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int ty = slot_ty(j);
      if (slot_on(j)) {
        const float vl = lastodd ? v[j].v[1] : v[j].v[0];  // column W - 1
        const float v0 = gx <= W - 1 ? v[j].v[0] : vl;
        const float v1 = gx + 1 <= W - 1 ? v[j].v[1] : vl;
        typedef float v2 __attribute__((ext_vector_type(2)));
        *(v2*)&t[ty][2 * q + 2] = v2{v0, v1};
      }
    }
  }
  if (threadIdx.x < 2 * TH) {
    // halo columns x0 - 1 and x0 + 64 (clamped: the mirror at the image edge)
    const int side = threadIdx.x / TH, ty = threadIdx.x - side * TH;
    const int hx = side == 0 ? max(x0 - 1, 0) : min(x0 + kTileW, W - 1);
    const int gy = min(max(y0 - 1 + ty, 0), H - 1);
    // (a prolongation's coarse patch covers the halo columns' stencils too)
    t[ty][side == 0 ? 1 : kTileW + 2] = F.value(F.col(hx), gy);
  }
  __syncthreads();
  const bool rest = mode_rest(MODE) && a.rest;
  __shared__ float rt[mode_rest(MODE) ? kTileH : 1][mode_rest(MODE) ? kTileW : 1];
  const Fld<TU> uo(a.u_out, (size_t)ch * lv.plane, a.s_u, a.rho, ch);
  const Fld<TU> ro(a.r, (size_t)ch * lv.plane, a.s_r, a.rho, ch);
  const Fld<TC> rlo(a.r, (size_t)ch * lv.plane, a.s_r, a.rho, ch);  // r_tc
  double acc = 0.0;
  if constexpr (mode_fin(MODE)) {
#pragma unroll
    for (int k = 0; k < RK; ++k) mk[k] = ld_mask2(a.c, min(y0 + g + NG * k, H - 1) * lv.P + gxe);
    if (!a.solution) {
#pragma unroll
      for (int k = 0; k < RK; ++k) bvv[k] = ld2(F.bb, min(y0 + g + NG * k, H - 1) * lv.P + gxe);
    } else {
#pragma unroll
      for (int k = 0; k < RK; ++k) bvv[k] = Px2{{0.0f, 0.0f}};
    }
  }
  const bool in0 = gx < W, in1 = gx + 1 < W;
  const bool r_small = mode_fin(MODE) || ((MODE == PASS_PSOL || MODE == PASS_RES) && a.r_tc);
#pragma unroll
  for (int k = 0; k < RK; ++k) {
    const int ty = g + NG * k;
    const int gy = y0 + ty;
    if (!(in0 && gy < H)) continue;
    const int off = gy * lv.P + gx;
    const float* row = &t[ty + 1][0];
    const float u0 = row[2 * q + 2], u1 = row[2 * q + 3];
    const float ul = row[2 * q + 1], ur = row[2 * q + 4];
    const float up0 = t[ty][2 * q + 2], up1 = t[ty][2 * q + 3];
    const float dn0 = t[ty + 2][2 * q + 2], dn1 = t[ty + 2][2 * q + 3];
    if constexpr (MODE != PASS_RES) {
      if (in1)
        st2(uo, off, u0, u1);
      else
        uo.st(off, u0);
    }
    double r[2];
    {
      const double nb0 = ((double)ul + (double)u1) + ((double)up0 + (double)dn0);
      const double nb1 = ((double)u0 + (double)ur) + ((double)up1 + (double)dn1);
      const bool kn0 = (mk[k] & 0xffu) != 0, kn1 = (mk[k] >> 8) != 0;
      const double b0 = bvv[k].v[0], b1 = bvv[k].v[1];
      if constexpr (MODE == PASS_RES) {
        r[0] = kn0 ? b0 - (double)u0 : b0 - fma(4.0, (double)u0, -nb0);
        r[1] = kn1 ? b1 - (double)u1 : b1 - fma(4.0, (double)u1, -nb1);
      } else {
        // Every pass but the residual-only one leaves u == b at known pixels, so
        // the residual there is exactly 0; and b is 0 at the unknown pixels of a
        // solution problem, so it is read only for correction problems.
        r[0] = kn0 ? 0.0 : b0 - fma(4.0, (double)u0, -nb0);
        r[1] = kn1 ? 0.0 : b1 - fma(4.0, (double)u1, -nb1);
      }
    }
    const float rf0 = (float)r[0], rf1 = (float)r[1];
    if constexpr (mode_rest(MODE)) {
      if (rest) {
        rt[ty][2 * q] = rf0;
        rt[ty][2 * q + 1] = rf1;
        continue;
      }
    }
    if (r_small) {
      if (in1)
        st2(rlo, off, rf0, rf1);
      else
        rlo.st(off, rf0);
    } else {
      if (in1)
        st2(ro, off, rf0, rf1);
      else
        ro.st(off, rf0);
    }
    acc += r[0] * r[0];
    if (in1) acc += r[1] * r[1];
  }
  if constexpr (mode_rest(MODE)) {
    if (rest) {
      // The tile's coarse cells have all their children inside the tile.
      __syncthreads();
      const LevelView& cl = a.clv;
      const Fld<TC> bco(a.bc, (size_t)ch * cl.plane, a.s_cr, a.rho, ch);
      const Fld<TC> rco(a.rc, (size_t)ch * cl.plane, a.s_cr, a.rho, ch);
      const Fld<TC> uco(a.uc0, (size_t)ch * cl.plane, a.s_cr, a.rho, ch);
      constexpr int CW = kTileW / 2, CH = kTileH / 2;
#pragma unroll
      for (int qq = threadIdx.x; qq < CW * CH; qq += kPassThreads) {
        const int X = (x0 >> 1) + (qq % CW), Y = (y0 >> 1) + (qq / CW);
        if (X < cl.W && Y < cl.H) {
          const int occ = Y * cl.P + X;
          double v = 0.0;
          if (!a.cc[occ]) {
            double sr = 0.0;
            int n = 0;
            for (int dy = 0; dy < 2; ++dy)
              for (int dx = 0; dx < 2; ++dx) {
                const int y = 2 * Y + dy, x = 2 * X + dx;
                if (y < H && x < W) {
                  sr += (double)rt[y - y0][x - x0];
                  ++n;
                }
              }
            v = 4.0 * sr / (double)n;
          }
          const float vf = (float)v;
          bco.st(occ, vf);
          uco.st(occ, 0.0f);
          rco.st(occ, vf);
          acc += (double)vf * (double)vf;
        }
      }
    }
  }
  reduce_norm(acc, ch, tile, ntiles, a.norm);
}

// ---------------------------------------------------------------------------
// plain conjugate gradients on the finest grid (comparison schedule)
// ---------------------------------------------------------------------------

// Direction pass over a 64x32 tile: p = r + beta p on the tile and a one-pixel
// halo (a halo pixel outside the image mirrors its neighbour, so the 5-point
// stencil sees the reflecting boundary), then q = A p at the tile's unknown
// pixels (0 at known ones), p.q per channel.
__device__ __forceinline__ void cg_dir_body(const CgArgs& a, unsigned lin) {
  constexpr int TW = kTileW + 2, TH = kTileH + 2;
  constexpr int NG = kPassThreads / kTileW;
  constexpr int RJ = (TH + NG - 1) / NG;
  constexpr int RK = kTileH / NG;
  const LevelView& lv = a.lv;
  const unsigned tiles_x = (unsigned)((lv.W + kTileW - 1) / kTileW);
  const unsigned ntiles = tiles_x * (unsigned)((lv.H + kTileH - 1) / kTileH);
  const int ch = lin / ntiles;
  const unsigned tile = lin - (unsigned)ch * ntiles;
  if (!channel_active(a.active, ch)) return;  // the whole workgroup: one channel
  const int x0 = (int)(tile % tiles_x) * kTileW, y0 = (int)(tile / tiles_x) * kTileH;
  __shared__ float t[TH][TW];
  const size_t po = (size_t)ch * lv.plane;
  const gptr<const float> r = glb((const float*)a.r + po);
  const gptr<const float> pin = glb((a.first ? (const float*)a.r : a.p_in) + po);
  // A level whose pixels are all known (coarse levels of a dense mask) has
  // r = 0 and r.r = 0: then beta = 0 keeps p = 0 instead of 0/0.
  const double rho_old = a.first ? 0.0 : glb(a.rho_old)[ch];
  const float beta = rho_old > 0.0 ? (float)(glb(a.rho)[ch] / rho_old) : 0.0f;
  const int c = threadIdx.x & (kTileW - 1), g = threadIdx.x / kTileW;
  const int gx = x0 + c, gxc = min(gx, lv.W - 1);
  uint8_t mk[RK];
#pragma unroll
  for (int k = 0; k < RK; ++k) mk[k] = glb(a.c)[min(y0 + g * RK + k, lv.H - 1) * lv.P + gxc];
  float rv[RJ], pv[RJ];
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int ty = min(g + NG * j, TH - 1);
    const int off = min(max(y0 - 1 + ty, 0), lv.H - 1) * lv.P + gxc;
    rv[j] = r[off];
    pv[j] = pin[off];
  }
  float hr = 0.0f, hp = 0.0f;
  const int side = threadIdx.x / TH, hty = threadIdx.x - side * TH;
  if (threadIdx.x < 2 * TH) {
    const int hx = side == 0 ? max(x0 - 1, 0) : min(x0 + kTileW, lv.W - 1);
    const int off = min(max(y0 - 1 + hty, 0), lv.H - 1) * lv.P + hx;
    hr = r[off];
    hp = pin[off];
  }
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int ty = g + NG * j;
    if (ty < TH) t[ty][c + 1] = a.first ? rv[j] : rv[j] + beta * pv[j];
  }
  if (threadIdx.x < 2 * TH) t[hty][side == 0 ? 0 : TW - 1] = a.first ? hr : hr + beta * hp;
  __syncthreads();
  const size_t base = po;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < RK; ++k) {
    const int ty = g * RK + k, gy = y0 + ty;
    if (gx < lv.W && gy < lv.H) {
      const float p = t[ty + 1][c + 1];
      const float nb = (t[ty + 1][c] + t[ty + 1][c + 2]) + (t[ty][c + 1] + t[ty + 2][c + 1]);
      const float q = mk[k] ? 0.0f : 4.0f * p - nb;
      const size_t off = base + (size_t)gy * lv.P + gx;
      glb(a.p_out)[off] = p;
      glb(a.q)[off] = q;
      acc += (double)p * (double)q;
    }
  }
  reduce_norm(acc, ch, tile, ntiles, a.norm);
}

// Step pass over the same tiles: x += alpha p, r -= alpha q, r.r per channel.
__device__ __forceinline__ void cg_step_body(const CgArgs& a, unsigned lin) {
  constexpr int NG = kPassThreads / kTileW;
  constexpr int RK = kTileH / NG;
  const LevelView& lv = a.lv;
  const unsigned tiles_x = (unsigned)((lv.W + kTileW - 1) / kTileW);
  const unsigned ntiles = tiles_x * (unsigned)((lv.H + kTileH - 1) / kTileH);
  const int ch = lin / ntiles;
  const unsigned tile = lin - (unsigned)ch * ntiles;
  if (!channel_active(a.active, ch)) return;  // the whole workgroup: one channel
  const int x0 = (int)(tile % tiles_x) * kTileW, y0 = (int)(tile / tiles_x) * kTileH;
  const int c = threadIdx.x & (kTileW - 1), g = threadIdx.x / kTileW;
  const int gx = x0 + c, gxc = min(gx, lv.W - 1);
  const size_t po = (size_t)ch * lv.plane;
  const gptr<float> x = glb(a.x + po), r = glb(a.r + po);
  const gptr<const float> p = glb(a.p_in + po), q = glb((const float*)a.q + po);
  const double pq = glb(a.pq)[ch];
  const float alpha = pq > 0.0 ? (float)(glb(a.rho)[ch] / pq) : 0.0f;
  float xv[RK], rv[RK], pv[RK], qv[RK];
#pragma unroll
  for (int k = 0; k < RK; ++k) {
    const int off = min(y0 + g * RK + k, lv.H - 1) * lv.P + gxc;
    xv[k] = x[off];
    rv[k] = r[off];
    pv[k] = p[off];
    qv[k] = q[off];
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < RK; ++k) {
    const int gy = y0 + g * RK + k;
    if (gx < lv.W && gy < lv.H) {
      const int off = gy * lv.P + gx;
      const float rn = rv[k] - alpha * qv[k];
      x[off] = xv[k] + alpha * pv[k];
      r[off] = rn;
      acc += (double)rn * (double)rn;
    }
  }
  reduce_norm(acc, ch, tile, ntiles, a.norm);
}

// ---------------------------------------------------------------------------
// residual restriction (Sections 4.1, 4.4)
// ---------------------------------------------------------------------------

template <class TF, class TC>
__device__ __forceinline__ void restrict_body(const RestrictArgs& a, unsigned lin) {
  const unsigned tiles_x = (unsigned)((a.cl.W + kTileW - 1) / kTileW);
  const unsigned ntiles = tiles_x * (unsigned)((a.cl.H + kTileH - 1) / kTileH);
  const int ch = lin / ntiles;
  const unsigned tile = lin - (unsigned)ch * ntiles;
  if (!channel_active(a.active, ch)) return;
  const LevelView& fl = a.fl;
  const LevelView& cl = a.cl;
  const int X = (int)(tile % tiles_x) * kTileW + (threadIdx.x & 63);
  const int Yb = (int)(tile / tiles_x) * kTileH + (threadIdx.x >> 6) * (kTileH / 4);
  double acc = 0.0;
  const Fld<TF> r(a.rf, (size_t)ch * fl.plane, a.s_rf, a.rho, ch);
  const Fld<TC> bc(a.bc, (size_t)ch * cl.plane, a.s_cr, a.rho, ch);
  const Fld<TC> uc(a.uc, (size_t)ch * cl.plane, a.s_cr, a.rho, ch);
  const Fld<TC> rc(a.rc, (size_t)ch * cl.plane, a.s_cr, a.rho, ch);
#pragma unroll
  for (int k = 0; k < kTileH / 4; ++k) {
    const int Y = Yb + k;
    if (X < cl.W && Y < cl.H) {
      const int oc = Y * cl.P + X;
      double v = 0.0;
      if (!a.cc[oc]) {
        double s = 0.0;
        int n = 0;
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            const int y = 2 * Y + dy, x = 2 * X + dx;
            if (y < fl.H && x < fl.W) { s += (double)r.ld(y * fl.P + x); ++n; }
          }
        v = 4.0 * s / (double)n;
      }
      const float vf = (float)v;
      bc.st(oc, vf);
      uc.st(oc, 0.0f);
      rc.st(oc, vf);
      acc += (double)vf * (double)vf;
    }
  }
  reduce_norm(acc, ch, tile, ntiles, a.norm);
}

// ---------------------------------------------------------------------------
// local CG on one block held in the registers of one wavefront
// ---------------------------------------------------------------------------
//
// Lane layout for block side B (B in {16, 32}; 64 is BlockCG64): lane = lx + B * g, where lx is
// the column inside the block and g one of G = 64 / B row groups; each lane
// holds the R = B / G rows g*R .. g*R + R - 1 of its column.  Horizontal
// neighbours come from lanes +-1 through DPP wave shifts; vertical neighbours
// are in the same lane's registers except across row groups (lanes +-B).
template <int B>
struct BlockCG {
  static constexpr int G = kWave / B;
  static constexpr int R = B / G;
  int lane, lx, g;
  float hasL, hasR;  // the lane to the left / right belongs to the same row group
  float dg[R];       // diagonal of A_i, 0 at known and outside pixels
  bool nm[R];        // unknown pixel of the block (held as lane masks in scalar registers)

  __device__ void apply(const float (&x)[R], float (&q)[R]) const {
    float fa = __shfl(x[R - 1], (lane - B) & 63);
    float fb = __shfl(x[0], (lane + B) & 63);
    fa = g > 0 ? fa : 0.0f;
    fb = g < G - 1 ? fb : 0.0f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const float l = lane_from_left(x[k]) * hasL;
      const float r = lane_from_right(x[k]) * hasR;
      const float up = k > 0 ? x[k - 1] : fa;
      const float dn = k < R - 1 ? x[k + 1] : fb;
      q[k] = nm[k] ? dg[k] * x[k] - ((l + r) + (up + dn)) : 0.0f;
    }
  }

  // Set up the lane geometry and the diagonal for a block at (x0, y0) of size
  // bw x bh on a W x H level.  A neighbour outside the block but inside the
  // image is a cut edge and adds gamma (Robin); one outside the image adds 0.
  __device__ void setup(int x0, int y0, int bw, int bh, int W, int H, float gamma,
                        const uint8_t* __restrict__ c, int P) {
    lane = threadIdx.x & 63;
    lx = lane % B;
    g = lane / B;
    hasL = lx > 0 ? 1.0f : 0.0f;
    hasR = lx < B - 1 ? 1.0f : 0.0f;
    const bool colok = lx < bw;
    const float dl = lx > 0 ? 1.0f : (x0 > 0 ? gamma : 0.0f);
    const float dr = lx < bw - 1 ? 1.0f : (x0 + bw < W ? gamma : 0.0f);
    // every lane loads, from a clamped in-block address, so that the loads
    // issue together instead of one branch (and one wait) per row
    const int cx = x0 + min(lx, bw - 1);
    uint8_t cm[R];
#pragma unroll
    for (int k = 0; k < R; ++k) cm[k] = glb(c)[(size_t)(y0 + min(g * R + k, bh - 1)) * P + cx];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int ly = g * R + k;
      const bool ok = colok && ly < bh;
      const bool unknown = ok & (cm[k] == 0);  // no short circuit: keeps every load unconditional
      const float du = ly > 0 ? 1.0f : (y0 > 0 ? gamma : 0.0f);
      const float dd = ly < bh - 1 ? 1.0f : (y0 + bh < H ? gamma : 0.0f);
      nm[k] = unknown;
      dg[k] = unknown ? (dl + dr) + (du + dd) : 0.0f;
    }
  }

  // Plain CG from v = 0 on A_i v = rho (rho is overwritten by the final
  // residual).  Stops when ||rho||^2 <= thr or after maxit iterations.
  __device__ int solve(float (&rho)[R], float (&v)[R], float thr, int maxit) const {
    float p[R], q[R];
    float rr = 0.0f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      rho[k] = nm[k] ? rho[k] : 0.0f;
      v[k] = 0.0f;
      p[k] = rho[k];
      rr += rho[k] * rho[k];
    }
    rr = wave_sum(rr);
    int it = 0;
    while (it < maxit && rr > thr && rr >= kTiny) {
      apply(p, q);
      float pq = 0.0f;
#pragma unroll
      for (int k = 0; k < R; ++k) pq += p[k] * q[k];
      pq = wave_sum(pq);
      if (!(pq >= kTiny)) break;
      const float alpha = rr * __builtin_amdgcn_rcpf(pq);  // CG needs no IEEE division
      float rn = 0.0f;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        v[k] += alpha * p[k];
        rho[k] -= alpha * q[k];
        rn += rho[k] * rho[k];
      }
      rn = wave_sum(rn);
      const float beta = rn * __builtin_amdgcn_rcpf(rr);
      rr = rn;
#pragma unroll
      for (int k = 0; k < R; ++k) p[k] = rho[k] + beta * p[k];
      ++it;
    }
    return it;
  }
};

// The local CG for B = 32 in float32 with two columns per lane: lane = c + 16 g
// holds columns 2c and 2c + 1 (index h = 0, 1) of rows 8g .. 8g + 7.  One
// block row then spans one 16-lane DPP row, whose shifts bring in 0 at the
// block's left and right edges by themselves, and both horizontal neighbours
// of a pixel cost one shifted add.  Arithmetic is that of BlockCG (same
// stencil evaluation order); only the order of the dot-product sums differs.
struct BlockCG2 {
  static constexpr int B = 32, C = 16, G = 4, R = 8;
  int lane, c, g;
  float dg[2][R];  // diagonal of A_i, 0 at known and outside pixels
  bool nm[2][R];   // unknown pixel of the block

  __device__ void apply(const float (&x)[2][R], float (&q)[2][R]) const {
    float ua = __shfl(x[0][R - 1], (lane - C) & 63), ub = __shfl(x[1][R - 1], (lane - C) & 63);
    float da = __shfl(x[0][0], (lane + C) & 63), db = __shfl(x[1][0], (lane + C) & 63);
    ua = g > 0 ? ua : 0.0f;
    ub = g > 0 ? ub : 0.0f;
    da = g < G - 1 ? da : 0.0f;
    db = g < G - 1 ? db : 0.0f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      // left and right of column 2c: column 2c + 1 of the lane to the left, own column 2c + 1
      const float ha = row_from_left(x[1][k]) + x[1][k];
      // left and right of column 2c + 1: own column 2c, column 2c of the lane to the right
      const float hb = x[0][k] + row_from_right(x[0][k]);
      const float upa = k > 0 ? x[0][k - 1] : ua, dna = k < R - 1 ? x[0][k + 1] : da;
      const float upb = k > 0 ? x[1][k - 1] : ub, dnb = k < R - 1 ? x[1][k + 1] : db;
      q[0][k] = nm[0][k] ? dg[0][k] * x[0][k] - (ha + (upa + dna)) : 0.0f;
      q[1][k] = nm[1][k] ? dg[1][k] * x[1][k] - (hb + (upb + dnb)) : 0.0f;
    }
  }

  // Lane geometry and diagonal for a block at (x0, y0) of size bw x bh on a
  // W x H level, as BlockCG::setup.
  __device__ void setup(int x0, int y0, int bw, int bh, int W, int H, float gamma,
                        const uint8_t* __restrict__ m, int P) {
    lane = threadIdx.x & 63;
    c = lane & (C - 1);
    g = lane / C;
    float dl[2], dr[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int lx = 2 * c + h;
      dl[h] = lx > 0 ? 1.0f : (x0 > 0 ? gamma : 0.0f);
      dr[h] = lx < bw - 1 ? 1.0f : (x0 + bw < W ? gamma : 0.0f);
    }
    // the lane's two columns as one 2-byte load (the block's last pair when
    // the lane lies past a clipped block: those pixels are not used)
    const int pe = x0 + min(2 * c, (bw - 1) & ~1);
    uint8_t cm[2][R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const unsigned row = (unsigned)(y0 + min(g * R + k, bh - 1)) * (unsigned)P;
      const unsigned short w = ld_mask2(m, (int)(row + pe));
      cm[0][k] = (uint8_t)(w & 0xffu);
      cm[1][k] = (uint8_t)(w >> 8);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int ly = g * R + k;
      const float du = ly > 0 ? 1.0f : (y0 > 0 ? gamma : 0.0f);
      const float dd = ly < bh - 1 ? 1.0f : (y0 + bh < H ? gamma : 0.0f);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool unknown = (2 * c + h < bw) & (ly < bh) & (cm[h][k] == 0);  // loads stay unconditional
        nm[h][k] = unknown;
        dg[h][k] = unknown ? (dl[h] + dr[h]) + (du + dd) : 0.0f;
      }
    }
  }

  // Plain CG from v = 0 on A_i v = rho (rho is overwritten by the final
  // residual).  Stops when ||rho||^2 <= thr or after maxit iterations.
  __device__ int solve(float (&rho)[2][R], float (&v)[2][R], float thr, int maxit) const {
    float p[2][R], q[2][R];
    float rr = 0.0f;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < R; ++k) {
        rho[h][k] = nm[h][k] ? rho[h][k] : 0.0f;
        v[h][k] = 0.0f;
        p[h][k] = rho[h][k];
        rr += rho[h][k] * rho[h][k];
      }
    rr = wave_sum(rr);
    int it = 0;
    while (it < maxit && rr > thr && rr >= kTiny) {
      apply(p, q);
      float pq = 0.0f;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < R; ++k) pq += p[h][k] * q[h][k];
      pq = wave_sum(pq);
      if (!(pq >= kTiny)) break;
      const float alpha = rr * __builtin_amdgcn_rcpf(pq);
      float rn = 0.0f;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < R; ++k) {
          v[h][k] += alpha * p[h][k];
          rho[h][k] -= alpha * q[h][k];
          rn += rho[h][k] * rho[h][k];
        }
      rn = wave_sum(rn);
      const float beta = rn * __builtin_amdgcn_rcpf(rr);
      rr = rn;
      // p = p * beta + rho in place: written as C++ the compiler copies rho,
      // accumulates with v_fmac and copies the result back (32 extra moves)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < R; ++k)
          asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(p[h][k]) : "v"(beta), "v"(rho[h][k]));
      ++it;
    }
    return it;
  }
};

// The local CG of the 16-bit forms (B = 32) in packed float16 arithmetic,
// in the BlockCG2 lane layout: a lane's two pixels of one row form one half2
// (low half: column 2c), so that one packed instruction works on both and
// vertical neighbours are whole registers of the same lane.  The right-hand
// side arrives normalised to unit norm (all values well inside the float16
// range); dot products accumulate in float32 (dot2) and so does the
// solution.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned h2_bits(half2_t v) { return __builtin_bit_cast(unsigned, v); }
__device__ __forceinline__ half2_t bits_h2(unsigned v) { return __builtin_bit_cast(half2_t, v); }

struct BlockCGh2 {
  static constexpr int B = 32, C = 16, G = 4, R = 8;
  int lane, c, g;
  half2_t dg[R];  // diagonal of A_i (0 at known and outside pixels)
  half2_t nm[R];  // 1 at unknown pixels of the block, else 0

  // as BlockCG2::setup
  __device__ void setup(int x0, int y0, int bw, int bh, int W, int H, float gamma,
                        const uint8_t* __restrict__ m, int P) {
    lane = threadIdx.x & 63;
    c = lane & (C - 1);
    g = lane / C;
    float dl[2], dr[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int lx = 2 * c + h;
      dl[h] = lx > 0 ? 1.0f : (x0 > 0 ? gamma : 0.0f);
      dr[h] = lx < bw - 1 ? 1.0f : (x0 + bw < W ? gamma : 0.0f);
    }
    // the lane's two columns as one 2-byte load (the block's last pair when
    // the lane lies past a clipped block: those pixels are not used)
    const int pe = x0 + min(2 * c, (bw - 1) & ~1);
    uint8_t cm[2][R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const unsigned row = (unsigned)(y0 + min(g * R + k, bh - 1)) * (unsigned)P;
      const unsigned short w = ld_mask2(m, (int)(row + pe));
      cm[0][k] = (uint8_t)(w & 0xffu);
      cm[1][k] = (uint8_t)(w >> 8);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int ly = g * R + k;
      const float du = ly > 0 ? 1.0f : (y0 > 0 ? gamma : 0.0f);
      const float dd = ly < bh - 1 ? 1.0f : (y0 + bh < H ? gamma : 0.0f);
      float d[2], n[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool unknown = (2 * c + h < bw) & (ly < bh) & (cm[h][k] == 0);  // loads stay unconditional
        n[h] = unknown ? 1.0f : 0.0f;
        d[h] = unknown ? (dl[h] + dr[h]) + (du + dd) : 0.0f;
      }
      dg[k] = half2_t{(_Float16)d[0], (_Float16)d[1]};
      nm[k] = half2_t{(_Float16)n[0], (_Float16)n[1]};
    }
  }

  __device__ void apply(const half2_t (&x)[R], half2_t (&q)[R]) const {
    unsigned fa = (unsigned)__shfl((int)h2_bits(x[R - 1]), (lane - C) & 63);
    unsigned fb = (unsigned)__shfl((int)h2_bits(x[0]), (lane + C) & 63);
    fa = g > 0 ? fa : 0u;
    fb = g < G - 1 ? fb : 0u;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const unsigned xb = h2_bits(x[k]);
      // row shifts: the pair of the lane to the left / right (0 past the block row)
      const unsigned lp = (unsigned)__builtin_amdgcn_update_dpp(0, (int)xb, 0x111, 0xf, 0xf, true);
      const unsigned rp = (unsigned)__builtin_amdgcn_update_dpp(0, (int)xb, 0x101, 0xf, 0xf, true);
      // (left of column 2c, right of column 2c + 1) + (right of 2c, left of 2c + 1)
      const half2_t h = bits_h2(__builtin_amdgcn_alignbit(rp, lp, 16)) +
                        __builtin_shufflevector(x[k], x[k], 1, 0);
      const half2_t up = k > 0 ? x[k - 1] : bits_h2(fa);
      const half2_t dn = k < R - 1 ? x[k + 1] : bits_h2(fb);
      q[k] = (dg[k] * x[k] - (h + (up + dn))) * nm[k];
    }
  }

  __device__ static float dot(const half2_t (&a)[R], const half2_t (&b)[R]) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < R; ++k) s = __builtin_amdgcn_fdot2(a[k], b[k], s, false);
    return wave_sum(s);
  }

  // CG from v = 0 on A_i v = r for a unit-norm r (0 at known pixels),
  // stopping when ||r||^2 <= t or after maxit iterations.  v accumulates in
  // packed float16 too (one packed FMA per pixel pair instead of two
  // conversions and two float32 FMAs: 24 of 155 instructions per iteration)
  // and is returned in float32; it is stored as a 16-bit correction anyway.
  __device__ int solve(half2_t (&r)[R], float (&v)[2][R], float t, int maxit) const {
    half2_t p[R], q[R], vh[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      vh[k] = half2_t{(_Float16)0.0f, (_Float16)0.0f};
      p[k] = r[k];
    }
    float rr = dot(r, r);
    int it = 0;
    bool stop = false;
    // one exit only: a breakdown (p.Ap not positive and normal) takes a zero
    // step and ends the loop at its head (a second exit makes the compiler
    // copy the float32 solution registers every iteration)
    while (!stop && it < maxit && rr > t && rr >= kTiny) {
      apply(p, q);
      const float pq = dot(p, q);
      stop = !(pq >= kTiny);
      const float alpha = stop ? 0.0f : rr * __builtin_amdgcn_rcpf(pq);  // no IEEE division
      const _Float16 ah = (_Float16)alpha;
      const half2_t a2 = half2_t{ah, ah};
#pragma unroll
      for (int k = 0; k < R; ++k) {
        vh[k] = vh[k] + a2 * p[k];
        r[k] = r[k] - a2 * q[k];
      }
      const float rn = dot(r, r);
      const float beta = rn * __builtin_amdgcn_rcpf(rr);
      rr = rn;
      const _Float16 bh = (_Float16)beta;
      const half2_t b2 = half2_t{bh, bh};
#pragma unroll
      for (int k = 0; k < R; ++k) p[k] = r[k] + b2 * p[k];
      it += stop ? 0 : 1;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      v[0][k] = (float)vh[k].x;
      v[1][k] = (float)vh[k].y;
    }
    return it;
  }
};

// The local CG for B = 64: four wavefronts per block.  Wave w holds rows
// 16w .. 16w + 15, lane = column, so horizontal neighbours are wave-wide DPP
// shifts (0 past the block's left and right edges) and vertical ones are the
// lane's own registers except across waves: each iteration every wave puts
// the first and last rows of the search direction in LDS for its neighbours.
// Dot products are wave sums added over the four waves in LDS (fixed order).
// Arithmetic per pixel is that of BlockCG; three workgroup barriers per
// iteration.
struct BlockCG64 {
  static constexpr int B = 64, NW = 4, R = B / NW;
  struct Shared {
    float edge[2][NW][2][B];  // [buffer][wave][first, last row][column]
    float dot[2][NW];         // [p.q, r.r][wave]
  };
  Shared* sh;
  int lane, w;
  float hasL, hasR;
  float dg[R];
  bool nm[R];

  __device__ void apply(const float (&x)[R], float (&q)[R], int buf) const {
    sh->edge[buf][w][0][lane] = x[0];
    sh->edge[buf][w][1][lane] = x[R - 1];
    __syncthreads();
    const float fa = w > 0 ? sh->edge[buf][w - 1][1][lane] : 0.0f;
    const float fb = w < NW - 1 ? sh->edge[buf][w + 1][0][lane] : 0.0f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const float l = lane_from_left(x[k]) * hasL;
      const float r = lane_from_right(x[k]) * hasR;
      const float up = k > 0 ? x[k - 1] : fa;
      const float dn = k < R - 1 ? x[k + 1] : fb;
      q[k] = nm[k] ? dg[k] * x[k] - ((l + r) + (up + dn)) : 0.0f;
    }
  }

  // the block-wide sum of a per-lane value (uniform result, same order everywhere)
  __device__ float block_sum(float v, int slot) const {
    v = wave_sum(v);
    if (lane == 0) sh->dot[slot][w] = v;
    __syncthreads();
    const float t = (sh->dot[slot][0] + sh->dot[slot][1]) + (sh->dot[slot][2] + sh->dot[slot][3]);
    return t;
  }

  __device__ void setup(Shared* s, int x0, int y0, int bw, int bh, int W, int H, float gamma,
                        const uint8_t* __restrict__ c, int P) {
    sh = s;
    lane = threadIdx.x & 63;
    w = threadIdx.x >> 6;
    hasL = lane > 0 ? 1.0f : 0.0f;
    hasR = lane < B - 1 ? 1.0f : 0.0f;
    const bool colok = lane < bw;
    const float dl = lane > 0 ? 1.0f : (x0 > 0 ? gamma : 0.0f);
    const float dr = lane < bw - 1 ? 1.0f : (x0 + bw < W ? gamma : 0.0f);
    const int cx = x0 + min(lane, bw - 1);
    uint8_t cm[R];
#pragma unroll
    for (int k = 0; k < R; ++k) cm[k] = glb(c)[(size_t)(y0 + min(w * R + k, bh - 1)) * P + cx];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int ly = w * R + k;
      const bool unknown = (colok & (ly < bh)) & (cm[k] == 0);
      const float du = ly > 0 ? 1.0f : (y0 > 0 ? gamma : 0.0f);
      const float dd = ly < bh - 1 ? 1.0f : (y0 + bh < H ? gamma : 0.0f);
      nm[k] = unknown;
      dg[k] = unknown ? (dl + dr) + (du + dd) : 0.0f;
    }
  }

  // Plain CG from v = 0 on A_i v = rho; stops when ||rho||^2 <= thr or after
  // maxit iterations (every wave takes the same decisions: the sums are uniform).
  __device__ int solve(float (&rho)[R], float (&v)[R], float thr, int maxit) const {
    float p[R], q[R];
    float rr = 0.0f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      rho[k] = nm[k] ? rho[k] : 0.0f;
      v[k] = 0.0f;
      p[k] = rho[k];
      rr += rho[k] * rho[k];
    }
    rr = block_sum(rr, 1);
    int it = 0;
    while (it < maxit && rr > thr && rr >= kTiny) {
      apply(p, q, it & 1);
      float pq = 0.0f;
#pragma unroll
      for (int k = 0; k < R; ++k) pq += p[k] * q[k];
      pq = block_sum(pq, 0);
      if (!(pq >= kTiny)) break;
      const float alpha = rr * __builtin_amdgcn_rcpf(pq);
      float rn = 0.0f;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        v[k] += alpha * p[k];
        rho[k] -= alpha * q[k];
        rn += rho[k] * rho[k];
      }
      rn = block_sum(rn, 1);
      const float beta = rn * __builtin_amdgcn_rcpf(rr);
      rr = rn;
#pragma unroll
      for (int k = 0; k < R; ++k) p[k] = rho[k] + beta * p[k];
      ++it;
    }
    return it;
  }
};

__device__ __forceinline__ float pou_weight(int l, int nb, int k, int B, int o, float inv_o1) {
  // 1-D partition of unity (Section 3.1): 0 at the outermost overlap pixel,
  // 1 at the innermost, linear in between; 1 away from overlaps.
  if (k > 0 && l < o) return (float)l * inv_o1;
  if (k < nb - 1 && l >= B - o) return (float)(B - 1 - l) * inv_o1;
  return 1.0f;
}

// Threshold of the local CG stop (Section 3.2): tau * ||r||^2 * |Omega_i| / N.
__device__ __forceinline__ float block_threshold(const BlockArgs& a, int ch, int bw, int bh) {
  const double frac = (double)(bw * bh) * a.inv_area;
  double sn;
  if (a.npart > 0) {
    // the norm's partials, one per workgroup of the pass that wrote r, added
    // in a fixed order
    // (at most kDeferParts of them: every load is issued before the first add)
    const gptr<const double> p = glb(a.snorm + (size_t)ch * a.pstride);
    const int lane = (int)(threadIdx.x & 63);
    double pv[kDeferParts / kWave];
#pragma unroll
    for (int j = 0; j < kDeferParts / kWave; ++j) pv[j] = p[min(lane + j * kWave, a.npart - 1)];
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kDeferParts / kWave; ++j) v += lane + j * kWave < a.npart ? pv[j] : 0.0;
    sn = wave_sum_d(v);
  } else {
    sn = glb(a.snorm)[ch];
  }
  return (float)((double)a.tau * sn * frac);
}

__device__ __forceinline__ void count_iterations(const BlockArgs& a, size_t ib, int it) {
  if (a.itot && (threadIdx.x & 63) == 0) {
    a.itot[ib] += it;
    a.imax[ib] = max(a.imax[ib], it);
  }
}

// float32 local problems of side 32: BlockCG2 lane layout
template <class TC>
__device__ __forceinline__ void block_body_f32(const BlockArgs& a, int ch, unsigned bi, unsigned nblk) {
  constexpr int B = 32, R = BlockCG2::R;
  const LevelView& lv = a.lv;
  const int S = B - lv.o;
  const int bx = bi % lv.nbx, by = bi / lv.nbx;
  const int x0 = bx * S, y0 = by * S;
  const int bw = min(B, lv.W - x0), bh = min(B, lv.H - y0);
  BlockCG2 cg;
  cg.setup(x0, y0, bw, bh, lv.W, lv.H, a.gamma, a.c, lv.P);
  float rho[2][R], v[2][R];
  {
    // pair loads (pixels outside the block are zeroed by the solve)
    const Fld<float> r(a.r, (size_t)ch * lv.plane, Sc{1.0f, 0}, a.rho, ch);
    const int pe = x0 + min(2 * cg.c, (bw - 1) & ~1);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const Px2 v = ld2(r, (y0 + min(cg.g * R + k, bh - 1)) * lv.P + pe);
      rho[0][k] = v.v[0];
      rho[1][k] = v.v[1];
    }
  }
  const float thr = block_threshold(a, ch, bw, bh);
  const int it = cg.solve(rho, v, thr, a.maxit);  // zeroes rho outside the block
  const Fld<TC> out(a.contrib, (size_t)ch * ((size_t)nblk * B * B) + (size_t)bi * B * B,
                    a.s_contrib, a.rho, ch);
  float wx[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) wx[h] = pou_weight(2 * cg.c + h, lv.nbx, bx, B, lv.o, a.inv_o1);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int ly = cg.g * R + k;
    if (ly >= bh) continue;
    const float wy = pou_weight(ly, lv.nby, by, B, lv.o, a.inv_o1);
    const float c0 = wx[0] * wy * v[0][k], c1 = wx[1] * wy * v[1][k];
    if (2 * cg.c + 1 < bw)
      st2(out, ly * B + 2 * cg.c, c0, c1);
    else if (2 * cg.c < bw)
      out.st(ly * B + 2 * cg.c, c0);
  }
  count_iterations(a, (size_t)ch * nblk + bi, it);
}

// Local problems of side 32 with 16-bit corrections: BlockCGh2 in packed float16
template <class TR, class TC>
__device__ __forceinline__ void block_body_h(const BlockArgs& a, int ch, unsigned bi, unsigned nblk) {
  constexpr int B = 32, R = BlockCGh2::R;
  const LevelView& lv = a.lv;
  const int S = B - lv.o;
  const int bx = bi % lv.nbx, by = bi / lv.nbx;
  const int x0 = bx * S, y0 = by * S;
  const int bw = min(B, lv.W - x0), bh = min(B, lv.H - y0);
  BlockCGh2 cg;
  cg.setup(x0, y0, bw, bh, lv.W, lv.H, a.gamma, a.c, lv.P);
  // the stored (scaled) residual values; the residual is rs * stored
  const Fld<TR> rf(a.r, (size_t)ch * lv.plane, a.s_r, a.rho, ch);
  float raw[2][R];
  {
    // pair loads of the stored values (unit scale: rs is applied below)
    const Fld<TR> r(a.r, (size_t)ch * lv.plane, Sc{1.0f, 0}, a.rho, ch);
    const int pe = x0 + min(2 * cg.c, (bw - 1) & ~1);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const Px2 v = ld2(r, (y0 + min(cg.g * R + k, bh - 1)) * lv.P + pe);
      raw[0][k] = v.v[0];
      raw[1][k] = v.v[1];
    }
  }
  float ss = 0.0f;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const bool rowin = cg.g * R + k < bh;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      raw[h][k] = rowin && 2 * cg.c + h < bw ? raw[h][k] : 0.0f;  // outside the block
      ss += raw[h][k] * raw[h][k];
    }
  }
  ss = wave_sum(ss);  // ||r||^2 / rs^2
  const float thr = block_threshold(a, ch, bw, bh);
  const float rs2 = rf.s * rf.s;
  float v[2][R];
  int it = 0;
  float un = 0.0f;  // ||r||; stays 0 (and v = 0) when the block needs no solve
  if (ss * rs2 > thr && a.maxit > 0) {
    const float sc = __builtin_amdgcn_rsqf(ss);  // unit-norm right-hand side
    half2_t rh[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rh[k] = half2_t{(_Float16)(raw[0][k] * sc), (_Float16)(raw[1][k] * sc)};
    it = cg.solve(rh, v, thr * sc * sc / rs2, a.maxit);
    un = ss * sc * rf.s;
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) v[0][k] = v[1][k] = 0.0f;
  }
  // contribution = PoU weights * ||r|| * v in the correction type and scale;
  // a lane's two pixels of a row are adjacent: one 32-bit store
  static_assert(sizeof(TC) == 2, "16-bit corrections");
  const Fld<TC> out(a.contrib, (size_t)ch * ((size_t)nblk * B * B) + (size_t)bi * B * B,
                    a.s_contrib, a.rho, ch);
  float wx[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    wx[h] = pou_weight(2 * cg.c + h, lv.nbx, bx, B, lv.o, a.inv_o1) * (un * out.inv);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int ly = cg.g * R + k;
    if (ly >= bh) continue;
    const float wy = pou_weight(ly, lv.nby, by, B, lv.o, a.inv_o1);
    const TC c0 = (TC)(wx[0] * wy * v[0][k]), c1 = (TC)(wx[1] * wy * v[1][k]);
    const int e = ly * B + 2 * cg.c;
    if (2 * cg.c + 1 < bw) {
      const unsigned pair = (unsigned)__builtin_bit_cast(unsigned short, c0) |
                            ((unsigned)__builtin_bit_cast(unsigned short, c1) << 16);
      *(gptr<unsigned>)(out.p + e) = pair;
    } else if (2 * cg.c < bw) {
      out.p[e] = c0;
    }
  }
  count_iterations(a, (size_t)ch * nblk + bi, it);
}

// Local problems of side 64: BlockCG64, four wavefronts per block (any
// residual and correction type, arithmetic in float32).
template <class TR, class TC>
__device__ __forceinline__ void block_body_64(const BlockArgs& a, int ch, unsigned bi, unsigned nblk) {
  constexpr int B = 64, R = BlockCG64::R;
  __shared__ BlockCG64::Shared sh;
  const LevelView& lv = a.lv;
  const int S = B - lv.o;
  const int bx = bi % lv.nbx, by = bi / lv.nbx;
  const int x0 = bx * S, y0 = by * S;
  const int bw = min(B, lv.W - x0), bh = min(B, lv.H - y0);
  BlockCG64 cg;
  cg.setup(&sh, x0, y0, bw, bh, lv.W, lv.H, a.gamma, a.c, lv.P);
  float rho[R], v[R];
  const Fld<TR> r(a.r, (size_t)ch * lv.plane, a.s_r, a.rho, ch);
  const bool colok = cg.lane < bw;
  {
    const int cx = x0 + min(cg.lane, bw - 1);
#pragma unroll
    for (int k = 0; k < R; ++k) rho[k] = r.ld((y0 + min(cg.w * R + k, bh - 1)) * lv.P + cx);
#pragma unroll
    for (int k = 0; k < R; ++k)
      if (!(colok && cg.w * R + k < bh)) rho[k] = 0.0f;
  }
  const float thr = block_threshold(a, ch, bw, bh);
  const int it = cg.solve(rho, v, thr, a.maxit);
  const Fld<TC> out(a.contrib, (size_t)ch * ((size_t)nblk * B * B) + (size_t)bi * B * B,
                    a.s_contrib, a.rho, ch);
  const float wx = pou_weight(cg.lane, lv.nbx, bx, B, lv.o, a.inv_o1);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int ly = cg.w * R + k;
    if (colok && ly < bh) out.st(ly * B + cg.lane, wx * pou_weight(ly, lv.nby, by, B, lv.o, a.inv_o1) * v[k]);
  }
  if (cg.w == 0) count_iterations(a, (size_t)ch * nblk + bi, it);
}

template <int B, class TR, class TC>
__device__ __forceinline__ void block_body(const BlockArgs& a, unsigned lin) {
  const unsigned nblk = (unsigned)a.lv.nbx * (unsigned)a.lv.nby;
  const int ch = lin / nblk;
  const unsigned bi = lin - (unsigned)ch * nblk;
  if (!channel_active(a.active, ch)) return;  // the whole workgroup: one channel
  if constexpr (B == 64) {
    block_body_64<TR, TC>(a, ch, bi, nblk);
    return;
  }
  if constexpr (B == 32) {
    // a correction stored in 16 bits is solved for in packed float16 (with
    // float32 accumulation), whatever the residual's type
    if constexpr (is_f32<TR>() && is_f32<TC>())
      block_body_f32<TC>(a, ch, bi, nblk);
    else
      block_body_h<TR, TC>(a, ch, bi, nblk);
    return;
  }
  const LevelView& lv = a.lv;
  const int S = B - lv.o;
  const int bx = bi % lv.nbx, by = bi / lv.nbx;
  const int x0 = bx * S, y0 = by * S;
  const int bw = min(B, lv.W - x0), bh = min(B, lv.H - y0);
  BlockCG<B> cg;
  cg.setup(x0, y0, bw, bh, lv.W, lv.H, a.gamma, a.c, lv.P);
  constexpr int R = BlockCG<B>::R;
  float rho[R], v[R];
  const Fld<TR> r(a.r, (size_t)ch * lv.plane, a.s_r, a.rho, ch);
  const bool colok = cg.lx < bw;
  {
    const int cx = x0 + min(cg.lx, bw - 1);
#pragma unroll
    for (int k = 0; k < R; ++k) rho[k] = r.ld((y0 + min(cg.g * R + k, bh - 1)) * lv.P + cx);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int ly = cg.g * R + k;
      if (!(colok && ly < bh)) rho[k] = 0.0f;
    }
  }
  const float thr = block_threshold(a, ch, bw, bh);
  const int it = cg.solve(rho, v, thr, a.maxit);
  const Fld<TC> out(a.contrib, (size_t)ch * ((size_t)nblk * B * B) + (size_t)bi * B * B,
                    a.s_contrib, a.rho, ch);
  const float wx = pou_weight(cg.lx, lv.nbx, bx, B, lv.o, a.inv_o1);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int ly = cg.g * R + k;
    if (colok && ly < bh) out.st(ly * B + cg.lx, wx * pou_weight(ly, lv.nby, by, B, lv.o, a.inv_o1) * v[k]);
  }
  count_iterations(a, (size_t)ch * nblk + bi, it);
}

// The coarsest grid is a single block.  Residual in float64 from u, then CG,
// then u += v.  One wavefront per channel.
template <int B, class T>
__device__ __forceinline__ void coarse_body(const CoarseArgs& a, unsigned lin) {
  const int ch = (int)lin;
  if (!channel_active(a.active, ch)) return;
  const LevelView& lv = a.lv;
  BlockCG<B> cg;
  cg.setup(0, 0, lv.W, lv.H, lv.W, lv.H, 0.0f, a.c, lv.P);
  constexpr int R = BlockCG<B>::R;
  const bool colok = cg.lx < lv.W;
  float u[R], bb[R], known[R];
  const Fld<T> bp(a.b, (size_t)ch * lv.plane, a.s_b, a.rho, ch);
  const Fld<T> up(a.u, (size_t)ch * lv.plane, a.s_u, a.rho, ch);
  // loads from clamped in-block addresses, issued together
  uint8_t cm[R];
  float uu[R];
  {
    const int cx = min(cg.lx, lv.W - 1);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int o = min(cg.g * R + k, lv.H - 1) * lv.P + cx;
      cm[k] = glb(a.c)[o];
      bb[k] = bp.ld(o);
      uu[k] = a.init ? 0.0f : up.ld(o);
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int ly = cg.g * R + k;
    const bool ok = colok && ly < lv.H;
    const bool kn = ok && cm[k] != 0;
    known[k] = kn ? 1.0f : 0.0f;
    bb[k] = ok ? bb[k] : 0.0f;
    u[k] = ok ? (a.init ? (kn ? bb[k] : 0.0f) : uu[k]) : 0.0f;
  }
  // residual r = b - A u (float64 arithmetic), 0 at known pixels
  float rho[R];
  {
    float fa = __shfl(u[R - 1], (cg.lane - B) & 63);
    float fb = __shfl(u[0], (cg.lane + B) & 63);
    fa = cg.g > 0 ? fa : 0.0f;
    fb = cg.g < BlockCG<B>::G - 1 ? fb : 0.0f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const double l = (double)(lane_from_left(u[k]) * cg.hasL);
      const double r = (double)(lane_from_right(u[k]) * cg.hasR);
      const double upv = k > 0 ? u[k - 1] : fa;
      const double dn = k < R - 1 ? u[k + 1] : fb;
      const double res = (double)bb[k] - ((double)cg.dg[k] * (double)u[k] - ((l + r) + (upv + dn)));
      rho[k] = cg.nm[k] ? (float)res : 0.0f;
    }
  }
  float rr0 = 0.0f;
#pragma unroll
  for (int k = 0; k < R; ++k) rr0 += rho[k] * rho[k];
  rr0 = wave_sum(rr0);
  float v[R];
  const int it = cg.solve(rho, v, a.rel_tol * rr0, a.maxit);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int ly = cg.g * R + k;
    if (colok && ly < lv.H) up.st(ly * lv.P + cg.lx, known[k] != 0.0f ? bb[k] : u[k] + v[k]);
  }
  (void)it;
}

// ---------------------------------------------------------------------------
// kernels: one problem per launch (k_*) and batches of problems (k_*_b)
// ---------------------------------------------------------------------------

#define INPAINT_BATCH_LOOKUP(ARGS_T)                          \
  const unsigned g = xcd_remap(blockIdx.x, gridDim.x);        \
  const int p = find_problem(start, n, g);                    \
  const ARGS_T a = args[p];                                   \
  const unsigned lin = g - start[p];

__global__ void __launch_bounds__(256) k_output(OutputArgs a) { output_body(a, xcd_remap(blockIdx.x, gridDim.x)); }
__global__ void __launch_bounds__(256) k_output_b(const OutputArgs* __restrict__ args,
                                                  const unsigned* __restrict__ start, int n) {
  // the arguments are read in place: a private copy of this struct (with its
  // pointer array) would live in scratch memory
  const unsigned g = xcd_remap(blockIdx.x, gridDim.x);
  const int p = find_problem(start, n, g);
  output_body(args[p], g - start[p]);
}


__global__ void __launch_bounds__(256) k_warm_b(const WarmArgs* __restrict__ args,
                                                const unsigned* __restrict__ start, int n) {
  const unsigned g = xcd_remap(blockIdx.x, gridDim.x);
  const int p = find_problem(start, n, g);
  warm_body(args[p], g - start[p]);
}

template <class TF, class TC>
__global__ void __launch_bounds__(256) k_rhs_down(RhsArgs a) {
  rhs_body<TF, TC>(a, xcd_remap(blockIdx.x, gridDim.x));
}
template <class TF, class TC>
__global__ void __launch_bounds__(256) k_rhs_b(const RhsArgs* __restrict__ args,
                                               const unsigned* __restrict__ start, int n) {
  INPAINT_BATCH_LOOKUP(RhsArgs)
  rhs_body<TF, TC>(a, lin);
}

__global__ void __launch_bounds__(kPassThreads) k_stage(StageArgs a) {
  stage_body(a, xcd_remap(blockIdx.x, gridDim.x));
}
__global__ void __launch_bounds__(kPassThreads) k_stage_b(const StageArgs* __restrict__ args,
                                                         const unsigned* __restrict__ start, int n) {
  INPAINT_BATCH_LOOKUP(StageArgs)
  stage_body(a, lin);
}

template <int MODE, class TU, class TC>
__global__ void __launch_bounds__(kPassThreads) k_pass(PassArgs a) {
  pass_body<MODE, TU, TC>(a, xcd_remap(blockIdx.x, gridDim.x));
}
template <int MODE, class TU, class TC>
__global__ void __launch_bounds__(kPassThreads) k_pass_b(const PassArgs* __restrict__ args,
                                                        const unsigned* __restrict__ start, int n) {
  INPAINT_BATCH_LOOKUP(PassArgs)
  pass_body<MODE, TU, TC>(a, lin);
}

template <class TF, class TC>
__global__ void __launch_bounds__(kPassThreads) k_restrict(RestrictArgs a) {
  restrict_body<TF, TC>(a, xcd_remap(blockIdx.x, gridDim.x));
}
template <class TF, class TC>
__global__ void __launch_bounds__(kPassThreads) k_restrict_b(const RestrictArgs* __restrict__ args,
                                                            const unsigned* __restrict__ start, int n) {
  INPAINT_BATCH_LOOKUP(RestrictArgs)
  restrict_body<TF, TC>(a, lin);
}

// Five wavefronts per SIMD (at most 96 registers; six for the packed float16
// solve, 80 registers) hide the latency of the cross-lane operations and the
// block loads better than the four a free register allocation gives.
template <class TR>
constexpr int block_waves() { return is_f32<TR>() ? 5 : 6; }

template <int B, class TR, class TC>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(block_waves<TR>(), 8)))
k_block_solve(BlockArgs a) {
  block_body<B, TR, TC>(a, xcd_remap(blockIdx.x, gridDim.x));
}
// side 64: one block per workgroup of four wavefronts
template <class TR, class TC>
__global__ void __launch_bounds__(4 * kWave) k_block_solve64(BlockArgs a) {
  block_body<64, TR, TC>(a, xcd_remap(blockIdx.x, gridDim.x));
}
template <class TR, class TC>
__global__ void __launch_bounds__(4 * kWave) k_block_b64(const BlockArgs* __restrict__ args,
                                                        const unsigned* __restrict__ start, int n) {
  INPAINT_BATCH_LOOKUP(BlockArgs)
  block_body<64, TR, TC>(a, lin);
}
template <int B, class TR, class TC>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(block_waves<TR>(), 8)))
k_block_b(const BlockArgs* __restrict__ args,
                                                   const unsigned* __restrict__ start, int n) {
  INPAINT_BATCH_LOOKUP(BlockArgs)
  block_body<B, TR, TC>(a, lin);
}

template <int B, class T>
__global__ void __launch_bounds__(kWave) k_coarse_solve(CoarseArgs a) {
  coarse_body<B, T>(a, blockIdx.x);
}
template <int B, class T>
__global__ void __launch_bounds__(kWave) k_coarse_b(const CoarseArgs* __restrict__ args,
                                                    const unsigned* __restrict__ start, int n) {
  const unsigned g = blockIdx.x;
  const int p = find_problem(start, n, g);
  const CoarseArgs a = args[p];
  coarse_body<B, T>(a, g - start[p]);
}

__global__ void __launch_bounds__(kPassThreads) k_cg_dir_b(const CgArgs* __restrict__ args,
                                                         const unsigned* __restrict__ start, int n) {
  INPAINT_BATCH_LOOKUP(CgArgs)
  cg_dir_body(a, lin);
}
__global__ void __launch_bounds__(kPassThreads) k_cg_step_b(const CgArgs* __restrict__ args,
                                                          const unsigned* __restrict__ start, int n) {
  INPAINT_BATCH_LOOKUP(CgArgs)
  cg_step_body(a, lin);
}

#undef INPAINT_BATCH_LOOKUP

dim3 px_grid(int W, int H) { return dim3((W + 63) / 64, (H + 3) / 4); }

}  // namespace

hipError_t launch_cg_stats(LevelView lv, const int* itot, const int* imax, int C,
                           unsigned long long* cgstat, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_stats, dim3(C), dim3(kPassThreads), 0, s, lv, itot, imax, cgstat);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

size_t prec_bytes(int prec) { return prec == PREC_F32 ? 4 : 2; }

size_t pass_tiles(const LevelView& lv) {
  return (size_t)((lv.W + kTileW - 1) / kTileW) * (size_t)((lv.H + kTileH - 1) / kTileH);
}

// ---------------------------------------------------------------------------
// work counts (workgroups per problem)
// ---------------------------------------------------------------------------

unsigned work_stage(const StageArgs& a) { return (unsigned)pass_tiles(a.lv) * (unsigned)a.C; }
unsigned work_rhs(const RhsArgs& a) { return px_groups(a.cl.W, a.cl.H); }
unsigned work_pass(const PassArgs& a, int C) { return (unsigned)pass_tiles(a.lv) * (unsigned)C; }
unsigned work_restrict(const RestrictArgs& a, int C) { return (unsigned)pass_tiles(a.cl) * (unsigned)C; }
unsigned work_block(const BlockArgs& a, int C) {
  return (unsigned)a.lv.nbx * (unsigned)a.lv.nby * (unsigned)C;
}
unsigned work_coarse(const CoarseArgs&, int C) { return (unsigned)C; }
unsigned work_output(const OutputArgs& a) {
  return (unsigned)((a.lv.W + 63) / 64) * (unsigned)((a.lv.H + 4 * kOutRows - 1) / (4 * kOutRows)) *
         (unsigned)a.C;
}

// ---------------------------------------------------------------------------
// single-problem launchers
// ---------------------------------------------------------------------------

hipError_t launch_stage(const float* f, const uint8_t* mask, int W, int H, int C, int Pf,
                        LevelView lv, uint8_t* c, float* b, float* u, int* status, NormOut den,
                        hipStream_t s) {
  const StageArgs a{f, mask, W, H, Pf, C, lv, c, b, u, status, den};
  hipLaunchKernelGGL(k_stage, dim3(work_stage(a)), dim3(kPassThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rhs_down(LevelView fine, const uint8_t* cf, const void* bf, LevelView coarse,
                           uint8_t* cc, void* bc, int C, int naive, int prec, int fine_f32,
                           hipStream_t s) {
  const RhsArgs a{fine, coarse, cf, bf, cc, bc, C, naive};
  return with_types(prec, fine_f32, [&](auto tf, auto tc) {
    using TF = typename decltype(tf)::type;
    using TC = typename decltype(tc)::type;
    hipLaunchKernelGGL((k_rhs_down<TF, TC>), dim3(work_rhs(a)), dim3(256), 0, s, a);
    return hipGetLastError();
  });
}

hipError_t launch_pass(int mode, const PassArgs& a, int C, hipStream_t s) {
  const dim3 grid(work_pass(a, C));
  return with_types(a.prec, a.level0, [&](auto tu, auto tc) {
    using TU = typename decltype(tu)::type;
    using TC = typename decltype(tc)::type;
    switch (mode) {
#define INPAINT_PASS_CASE(M) \
  case M: hipLaunchKernelGGL((k_pass<M, TU, TC>), grid, dim3(kPassThreads), 0, s, a); break;
      INPAINT_PASS_CASE(PASS_RES)
      INPAINT_PASS_CASE(PASS_UPD)
      INPAINT_PASS_CASE(PASS_PSOL)
      INPAINT_PASS_CASE(PASS_PCORR)
      INPAINT_PASS_CASE(PASS_UPD0)
      INPAINT_PASS_CASE(PASS_FIN)
      INPAINT_PASS_CASE(PASS_FIN0)
      INPAINT_PASS_CASE(PASS_PCORR0)
#undef INPAINT_PASS_CASE
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t launch_restrict(const RestrictArgs& a, int C, hipStream_t s) {
  return with_types(a.prec, a.level0, [&](auto tf, auto tc) {
    using TF = typename decltype(tf)::type;
    using TC = typename decltype(tc)::type;
    hipLaunchKernelGGL((k_restrict<TF, TC>), dim3(work_restrict(a, C)), dim3(kPassThreads), 0, s, a);
    return hipGetLastError();
  });
}

hipError_t launch_block_solve(const BlockArgs& a, int C, hipStream_t s) {
  const dim3 grid(work_block(a, C));
  return with_types(a.prec, a.level0, [&](auto tr, auto tc) {
    using TR = typename decltype(tr)::type;
    using TC = typename decltype(tc)::type;
    if (a.lv.B == 32)
      hipLaunchKernelGGL((k_block_solve<32, TR, TC>), grid, dim3(kWave), 0, s, a);
    else if (a.lv.B == 64)
      hipLaunchKernelGGL((k_block_solve64<TR, TC>), grid, dim3(4 * kWave), 0, s, a);
    else if (a.lv.B == 16)
      hipLaunchKernelGGL((k_block_solve<16, TR, TC>), grid, dim3(kWave), 0, s, a);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  });
}

hipError_t launch_coarse_solve(const CoarseArgs& a, int C, hipStream_t s) {
  // the coarsest grid of a side-64 hierarchy is at most 32 x 32 (one wavefront)
  const int cb = a.lv.B == 64 ? 32 : a.lv.B;
  if (a.lv.W > cb || a.lv.H > cb) return hipErrorInvalidValue;
  return with_types(a.prec, a.level0, [&](auto tu, auto) {
    using T = typename decltype(tu)::type;
    if (cb == 32)
      hipLaunchKernelGGL((k_coarse_solve<32, T>), dim3(C), dim3(kWave), 0, s, a);
    else if (cb == 16)
      hipLaunchKernelGGL((k_coarse_solve<16, T>), dim3(C), dim3(kWave), 0, s, a);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  });
}

hipError_t launch_output(LevelView lv, const uint8_t* c, const float* b, const float* const* u_sel,
                         float* out, int Pout, int C, hipStream_t s) {
  OutputArgs a{};
  a.lv = lv;
  a.c = c;
  a.b = b;
  for (int ch = 0; ch < kMaxChannels; ++ch) a.u[ch] = u_sel[ch < C ? ch : 0];
  a.out = out;
  a.Pout = Pout;
  a.C = C;
  hipLaunchKernelGGL(k_output, dim3(work_output(a)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched launchers
// ---------------------------------------------------------------------------

hipError_t launch_stage_b(const StageArgs* args, const unsigned* start, int n, unsigned total,
                          hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stage_b, dim3(total), dim3(kPassThreads), 0, s, args, start, n);
  return hipGetLastError();
}

hipError_t launch_rhs_b(const RhsArgs* args, const unsigned* start, int n, unsigned total, int prec,
                        int fine_f32, hipStream_t s) {
  if (total == 0) return hipSuccess;
  return with_types(prec, fine_f32, [&](auto tf, auto tc) {
    using TF = typename decltype(tf)::type;
    using TC = typename decltype(tc)::type;
    hipLaunchKernelGGL((k_rhs_b<TF, TC>), dim3(total), dim3(256), 0, s, args, start, n);
    return hipGetLastError();
  });
}

hipError_t launch_pass_b(int mode, const PassArgs* args, const unsigned* start, int n,
                         unsigned total, int prec, int level0, hipStream_t s) {
  if (total == 0) return hipSuccess;
  const dim3 grid(total);
  return with_types(prec, level0, [&](auto tu, auto tc) {
    using TU = typename decltype(tu)::type;
    using TC = typename decltype(tc)::type;
    switch (mode) {
#define INPAINT_PASS_CASE(M)                                                                \
  case M:                                                                                   \
    hipLaunchKernelGGL((k_pass_b<M, TU, TC>), grid, dim3(kPassThreads), 0, s, args, start, n); \
    break;
      INPAINT_PASS_CASE(PASS_RES)
      INPAINT_PASS_CASE(PASS_UPD)
      INPAINT_PASS_CASE(PASS_PSOL)
      INPAINT_PASS_CASE(PASS_PCORR)
      INPAINT_PASS_CASE(PASS_UPD0)
      INPAINT_PASS_CASE(PASS_FIN)
      INPAINT_PASS_CASE(PASS_FIN0)
      INPAINT_PASS_CASE(PASS_PCORR0)
#undef INPAINT_PASS_CASE
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t launch_restrict_b(const RestrictArgs* args, const unsigned* start, int n, unsigned total,
                             int prec, int level0, hipStream_t s) {
  if (total == 0) return hipSuccess;
  return with_types(prec, level0, [&](auto tf, auto tc) {
    using TF = typename decltype(tf)::type;
    using TC = typename decltype(tc)::type;
    hipLaunchKernelGGL((k_restrict_b<TF, TC>), dim3(total), dim3(kPassThreads), 0, s, args, start, n);
    return hipGetLastError();
  });
}

hipError_t launch_block_b(const BlockArgs* args, const unsigned* start, int n, unsigned total,
                          int prec, int level0, int B, hipStream_t s) {
  if (total == 0) return hipSuccess;
  return with_types(prec, level0, [&](auto tr, auto tc) {
    using TR = typename decltype(tr)::type;
    using TC = typename decltype(tc)::type;
    if (B == 32)
      hipLaunchKernelGGL((k_block_b<32, TR, TC>), dim3(total), dim3(kWave), 0, s, args, start, n);
    else if (B == 64)
      hipLaunchKernelGGL((k_block_b64<TR, TC>), dim3(total), dim3(4 * kWave), 0, s, args, start, n);
    else if (B == 16)
      hipLaunchKernelGGL((k_block_b<16, TR, TC>), dim3(total), dim3(kWave), 0, s, args, start, n);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  });
}

hipError_t launch_coarse_b(const CoarseArgs* args, const unsigned* start, int n, unsigned total,
                           int prec, int level0, int B, hipStream_t s) {
  if (total == 0) return hipSuccess;
  if (B == 64) B = 32;  // the coarsest grid of a side-64 hierarchy is at most 32 x 32
  return with_types(prec, level0, [&](auto tu, auto) {
    using T = typename decltype(tu)::type;
    if (B == 32)
      hipLaunchKernelGGL((k_coarse_b<32, T>), dim3(total), dim3(kWave), 0, s, args, start, n);
    else if (B == 16)
      hipLaunchKernelGGL((k_coarse_b<16, T>), dim3(total), dim3(kWave), 0, s, args, start, n);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  });
}

hipError_t launch_output_b(const OutputArgs* args, const unsigned* start, int n, unsigned total,
                           hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_output_b, dim3(total), dim3(256), 0, s, args, start, n);
  return hipGetLastError();
}

unsigned work_warm(const WarmArgs& a) {
  return (unsigned)((a.lv.W + 63) / 64) * (unsigned)((a.lv.H + 4 * kOutRows - 1) / (4 * kOutRows)) *
         (unsigned)a.C;
}

hipError_t launch_warm_b(const WarmArgs* args, const unsigned* start, int n, unsigned total,
                         hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_warm_b, dim3(total), dim3(256), 0, s, args, start, n);
  return hipGetLastError();
}

unsigned work_cg(const CgArgs& a, int C) { return (unsigned)pass_tiles(a.lv) * (unsigned)C; }

hipError_t launch_cg_dir_b(const CgArgs* args, const unsigned* start, int n, unsigned total,
                           hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_dir_b, dim3(total), dim3(kPassThreads), 0, s, args, start, n);
  return hipGetLastError();
}

hipError_t launch_cg_step_b(const CgArgs* args, const unsigned* start, int n, unsigned total,
                            hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_step_b, dim3(total), dim3(kPassThreads), 0, s, args, start, n);
  return hipGetLastError();
}

}  // namespace inpaint
