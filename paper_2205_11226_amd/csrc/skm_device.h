// Device helpers shared by the estimation kernel and the HQL kernel: wave
// reductions, the per-block LDS layout, and the phases that stage a block's
// search window and find its admissible candidates with exact distances.
#pragma once

#include <limits.h>
#include <math.h>

#include "skm_internal.h"

namespace skm {

// ------------------------------------------------------------ wave helpers

// Workgroups are dispatched round-robin to the 8 XCDs.  xcd_block maps a
// workgroup id to an item index so that XCD x takes the x-th contiguous
// eighth of [0, n); the grid must hold at least 8 * ceil(n / 8) workgroups.
// Returns -1 for workgroups without an item.
static __device__ __forceinline__ int xcd_block(int wg, int n) {
  const int per = (n + 7) >> 3;
  const int i = (wg & 7) * per + (wg >> 3);
  return ((wg >> 3) < per && i < n) ? i : -1;
}

// Batched kernels: frame of item (or workgroup) g, the largest f with
// begin[f] <= g (begin is non-decreasing with begin[0] = 0).
static __device__ __forceinline__ int frame_of(const int* begin, int nf, int g) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static __device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

static __device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

template <typename T>
static __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
static __device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Full-wave reductions on DPP lane moves (no LDS traffic): every lane of the
// wave must be active.  Quad swaps, half-row and row mirrors leave each
// 16-lane row holding its sum; two row broadcasts carry the rows into lane 63,
// whose value is returned to all lanes.  The order is fixed.
template <int CTRL, int ROWS>
static __device__ __forceinline__ int dpp_i32(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
static __device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i32<CTRL, ROWS>(0, (int)(b & 0xffffffffll));
  const int hi = dpp_i32<CTRL, ROWS>(0, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
static __device__ __forceinline__ int wave_sum_full(int v) {
  v += dpp_i32<0xB1, 0xf>(0, v);     // quad_perm [1,0,3,2]
  v += dpp_i32<0x4E, 0xf>(0, v);     // quad_perm [2,3,0,1]
  v += dpp_i32<0x141, 0xf>(0, v);    // row_half_mirror
  v += dpp_i32<0x140, 0xf>(0, v);    // row_mirror
  v += dpp_i32<0x142, 0xa>(0, v);    // row_bcast:15 into rows 1, 3
  v += dpp_i32<0x143, 0xc>(0, v);    // row_bcast:31 into rows 2, 3
  return __builtin_amdgcn_readlane(v, 63);
}
// value of lane `l` (wave-uniform) in every lane
static __device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// inclusive prefix sum across the wave (row shifts, then row broadcasts)
static __device__ __forceinline__ int wave_incl_scan(int v) {
  v += dpp_i32<0x111, 0xf>(0, v);    // row_shr:1
  v += dpp_i32<0x112, 0xf>(0, v);    // row_shr:2
  v += dpp_i32<0x114, 0xf>(0, v);    // row_shr:4
  v += dpp_i32<0x118, 0xf>(0, v);    // row_shr:8
  v += dpp_i32<0x142, 0xa>(0, v);    // row_bcast:15 into rows 1, 3
  v += dpp_i32<0x143, 0xc>(0, v);    // row_bcast:31 into rows 2, 3
  return v;
}
static __device__ __forceinline__ double wave_sum_full(double v) {
  v += dpp_f64<0xB1, 0xf>(v);
  v += dpp_f64<0x4E, 0xf>(v);
  v += dpp_f64<0x141, 0xf>(v);
  v += dpp_f64<0x140, 0xf>(v);
  v += dpp_f64<0x142, 0xa>(v);
  v += dpp_f64<0x143, 0xc>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The same reductions for the common 32-bit types and doubles (the shuffle
// template above stays for 64-bit integers); every lane gets the result.
static __device__ __forceinline__ int wave_sum(int v) { return wave_sum_full(v); }
static __device__ __forceinline__ double wave_sum(double v) { return wave_sum_full(v); }
static __device__ __forceinline__ float wave_sum(float v) {
  v += __int_as_float(dpp_i32<0xB1, 0xf>(0, __float_as_int(v)));
  v += __int_as_float(dpp_i32<0x4E, 0xf>(0, __float_as_int(v)));
  v += __int_as_float(dpp_i32<0x141, 0xf>(0, __float_as_int(v)));
  v += __int_as_float(dpp_i32<0x140, 0xf>(0, __float_as_int(v)));
  v += __int_as_float(dpp_i32<0x142, 0xa>(0, __float_as_int(v)));
  v += __int_as_float(dpp_i32<0x143, 0xc>(0, __float_as_int(v)));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
// masked-off rows of the broadcasts read `old`: the neutral element
static __device__ __forceinline__ int wave_max(int v) {
  v = max(v, dpp_i32<0xB1, 0xf>(v, v));
  v = max(v, dpp_i32<0x4E, 0xf>(v, v));
  v = max(v, dpp_i32<0x141, 0xf>(v, v));
  v = max(v, dpp_i32<0x140, 0xf>(v, v));
  v = max(v, dpp_i32<0x142, 0xa>(INT_MIN, v));
  v = max(v, dpp_i32<0x143, 0xc>(INT_MIN, v));
  return __builtin_amdgcn_readlane(v, 63);
}
static __device__ __forceinline__ int wave_min(int v) {
  v = min(v, dpp_i32<0xB1, 0xf>(v, v));
  v = min(v, dpp_i32<0x4E, 0xf>(v, v));
  v = min(v, dpp_i32<0x141, 0xf>(v, v));
  v = min(v, dpp_i32<0x140, 0xf>(v, v));
  v = min(v, dpp_i32<0x142, 0xa>(INT_MAX, v));
  v = min(v, dpp_i32<0x143, 0xc>(INT_MAX, v));
  return __builtin_amdgcn_readlane(v, 63);
}

// Merge (m2, s2) into (m, s), both "max and sum of exp(x - max)".  Callers fix
// the merge order, so results are deterministic.
static __device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2) {
  if (m2 == -INFINITY) return;
  if (m == -INFINITY) { m = m2; s = s2; return; }
  if (m2 > m) { s = s * exp(m - m2) + s2; m = m2; }
  else        { s = s + s2 * exp(m2 - m); }
}

// 128-bit logical right shift of (lo, hi), 0 <= s < 128
static __device__ __forceinline__ void shr128(uint64_t lo, uint64_t hi, int s, uint64_t& olo,
                                              uint64_t& ohi) {
  if (s == 0) { olo = lo; ohi = hi; }
  else if (s < 64) { olo = (lo >> s) | (hi << (64 - s)); ohi = hi >> s; }
  else { olo = hi >> (s - 64); ohi = 0; }
}

// Adds a workgroup's (blocks with |m0| >= r B, largest |m0|) to the round's
// context rule (thread 0 calls it).  Only "some block is eligible" and, when
// none is, the largest |m0| matter, so the field is read first and the
// device-scope atomic is skipped when it would change nothing: after the
// first few workgroups, most do no atomic at all.
static __device__ __forceinline__ void note_context_rule(RoundState* st, int nq, int mx) {
  if (nq > 0) {
    if (__hip_atomic_load(&st->ctx_nq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      atomicMax(&st->ctx_nq, 1);
  } else if (mx > 0) {
    if (__hip_atomic_load(&st->ctx_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < mx)
      atomicMax(&st->ctx_max, mx);
  }
}

// ------------------------------------------------------------ LDS layout
//
// Per-block LDS carve-up (dynamic).  MC bounds the number of admissible
// candidates: a prototype can never overlap the block itself, so
// MC = (2W+1)^2 - (2 min(B-1, W) + 1)^2.  NU counts ring "units":
// horizontally adjacent pairs of ring pixels, or a single pixel with a dummy
// partner.
//   ell     f64 [MC]      log raw IDL weight of each candidate, -inf if dropped
//   cand    u32 [MC]      admissible candidates in raster order:
//                         window offset | bucket << 16 | radius << 24
//   selw    f32 [MC]      FP32 weights exp(ell - max) of the selected candidates
//   selo    u16 [MC]      their window offsets
//   qu      u32x2 [NU32]  per unit: packed int16 context pair, footprint offset;
//                         the ring units, then (for a block holding received
//                         pixels) its own B x B / 2 pairs, padded to a
//                         multiple of 32 with unknown pairs
//   utab    u32 [NU]      fixed unit table: footprint offset | single << 16
//   rowbits u64 [Wd][2]   availability bits of each window row
//   runbits u64 [Wd][2]   bit c set iff columns c .. c+B-1 are all available
//   cmask   u64 [D2][2]   bit dx of displacement row dy set iff the B x B
//                         prototype at (dy, dx) is admissible
//   winp    u32 [Wd*Wp]   window pixel pairs: int16 pixel | next pixel << 16,
//                         -1 = unknown (lost or out of frame); Wd rows of
//                         pitch Wp (odd), the padding column never read

struct MainLds {
  double* ell;
  uint32_t* cand;
  float* selw;
  uint16_t* selo;
  uint2* qu;
  uint32_t* utab;
  uint64_t* rowbits;
  uint64_t* runbits;
  uint64_t* cmask;
  uint32_t* winp;
};

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
__host__ __device__ inline int align32(int v) { return (v + 31) & ~31; }

__host__ __device__ inline size_t main_lds_layout(const DevParams& p, size_t* offs) {
  const size_t D2 = 2 * p.W + 1;
  size_t o = 0;
  offs[0] = o; o = align_up(o + sizeof(double) * p.MC, 16);
  offs[1] = o; o = align_up(o + sizeof(uint32_t) * p.MC, 16);
  offs[2] = o; o = align_up(o + sizeof(float) * p.MC, 16);
  offs[3] = o; o = align_up(o + sizeof(uint16_t) * p.MC, 16);
  offs[4] = o; o = align_up(o + sizeof(uint2) * (p.NR + p.B * p.B / 2 + 32), 16);   // + own, padded
  offs[5] = o; o = align_up(o + sizeof(uint32_t) * p.NR, 16);
  offs[6] = o; o = align_up(o + sizeof(uint64_t) * 2 * p.Wd, 16);
  offs[7] = o; o = align_up(o + sizeof(uint64_t) * 2 * p.Wd, 16);
  offs[8] = o; o = align_up(o + sizeof(uint64_t) * 2 * (2 * p.W + 1), 16);
  offs[9] = o; o = align_up(o + sizeof(uint32_t) * p.Wd * p.Wp, 16);
  return o;
}

static __device__ __forceinline__ MainLds carve_main_lds(unsigned char* raw, const DevParams& p) {
  size_t offs[10];
  main_lds_layout(p, offs);
  MainLds L;
  L.ell = (double*)(raw + offs[0]);
  L.cand = (uint32_t*)(raw + offs[1]);
  L.selw = (float*)(raw + offs[2]);
  L.selo = (uint16_t*)(raw + offs[3]);
  L.qu = (uint2*)(raw + offs[4]);
  L.utab = (uint32_t*)(raw + offs[5]);
  L.rowbits = (uint64_t*)(raw + offs[6]);
  L.runbits = (uint64_t*)(raw + offs[7]);
  L.cmask = (uint64_t*)(raw + offs[8]);
  L.winp = (uint32_t*)(raw + offs[9]);
  return L;
}

// Candidate word written by phase_candidates: window offset of the
// prototype's footprint origin (14 bits) | expansion bucket << 14 (4 bits);
// the estimation kernel adds the known-pair count n << 18 (10 bits).
static __device__ __forceinline__ int cand_off(uint32_t c) { return (int)(c & 0x3fffu); }
static __device__ __forceinline__ int cand_bucket(uint32_t c) { return (int)((c >> 14) & 0xfu); }
static __device__ __forceinline__ int cand_n(uint32_t c) { return (int)(c >> 18); }

// Estimation-kernel LDS (one block per workgroup), smaller than MainLds so
// that four workgroups fit a CU at the default geometry:
//   winp    u32 [Wd*Wp]   as in MainLds
//   qu      u32x2 [NR+B*B/2+32] as in MainLds
//   utab    u32 [NR]      as in MainLds
//   cand    u32 [MC+16]   candidate words; n added by the distance step
//   dist    u32 [MC]      exact distance d (~0u = dropped).  Before the
//                         distance step it holds rowbits, runbits and cmask.
//   sel     u32x2         after the weights step, cand and dist together
//                         hold the selected (window offset, FP32 weight)
//                         pairs, padded to a multiple of 8 with weight-0
//                         copies of the last pair's offset
//   part    f32 [2*kThreads] cross-group sums of the weighted average;
//                         aliases qu and utab when they are large enough
struct EstLds {
  uint32_t* winp;
  uint2* qu;
  uint32_t* utab;
  uint32_t* cand;
  uint32_t* dist;
  uint2* sel;
  float* part;
  MainLds m;          // view for the shared phases (ell, selw, selo unused)
};

__host__ __device__ inline size_t est_lds_layout(const DevParams& p, size_t* offs) {
  size_t o = 0;
  offs[0] = o; o = align_up(o + sizeof(uint32_t) * p.Wd * p.Wp, 16);
  offs[1] = o; o = align_up(o + sizeof(uint2) * (p.NR + p.B * p.B / 2 + 32), 16);
  offs[2] = o; o = align_up(o + sizeof(uint32_t) * p.NR, 16);
  const size_t qu_utab = o - offs[1];
  offs[3] = o; o = align_up(o + sizeof(uint32_t) * (p.MC + 16), 16);
  offs[4] = o;                                       // contiguous with cand
  const size_t bits = sizeof(uint64_t) * 2 * (2 * p.Wd + 2 * p.W + 1);
  const size_t dist = sizeof(uint32_t) * p.MC;
  o = align_up(o + (dist > bits ? dist : bits), 16);
  offs[5] = offs[1];
  const size_t part = sizeof(float) * 2 * kThreads;
  if (part > qu_utab) { offs[5] = o; o = align_up(o + part, 16); }
  return o;
}

static __device__ __forceinline__ EstLds carve_est_lds(unsigned char* raw, const DevParams& p) {
  size_t offs[6];
  est_lds_layout(p, offs);
  EstLds E;
  E.winp = (uint32_t*)(raw + offs[0]);
  E.qu = (uint2*)(raw + offs[1]);
  E.utab = (uint32_t*)(raw + offs[2]);
  E.cand = (uint32_t*)(raw + offs[3]);
  E.dist = (uint32_t*)(raw + offs[4]);
  E.sel = (uint2*)(raw + offs[3]);
  E.part = (float*)(raw + offs[5]);
  E.m.ell = nullptr;
  E.m.selw = nullptr;
  E.m.selo = nullptr;
  E.m.cand = E.cand;
  E.m.qu = E.qu;
  E.m.utab = E.utab;
  E.m.winp = E.winp;
  E.m.rowbits = (uint64_t*)E.dist;
  E.m.runbits = E.m.rowbits + 2 * p.Wd;
  E.m.cmask = E.m.runbits + 2 * p.Wd;
  return E;
}

// Small per-block values shared by the workgroup.
struct BlockShared {
  int NU, M, n_sel;
  int layer, radius_idx, flags, n_cand, n_complete;
  double lnu, den, xs;       // xs = 2^24 / den scales the weighted sums
  int red_i[kThreads / 64][4];
  int scan[kThreads / 64];
  unsigned long long bmax[kMaxRadii];
  int bcnt[kMaxRadii];
  double fsc[kMaxRadii];
  double ps[kThreads / 64][kMaxRadii];
  int rowbase[2 * kMaxWin + 1];
};

typedef short short2v __attribute__((ext_vector_type(2)));

// exclusive scan of one int per thread over the workgroup (fixed order)
static __device__ __forceinline__ int block_excl_scan(int v, int* s_w, int* total) {
  const int lane = lane_id(), wave = wave_id();
  const int x = wave_incl_scan(v);
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  int base = 0, tot = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wave) base += s_w[w];
    tot += s_w[w];
  }
  *total = tot;
  __syncthreads();
  return base + x - v;
}

// Sum of (q - p)^2 over both halves of two packed int16 pairs where neither
// half is negative (unknown), and the count of such halves, accumulated.
static __device__ __forceinline__ void pair_dist(uint32_t q, uint32_t pp, int& d, uint32_t& nacc) {
  const short2v qa = __builtin_bit_cast(short2v, q), pa = __builtin_bit_cast(short2v, pp);
  const short2v sgn = (qa | pa) >> (short2v){15, 15};          // 0xffff where unknown
  const uint32_t bad = __builtin_bit_cast(uint32_t, sgn);
  const uint32_t df = __builtin_bit_cast(uint32_t, (short2v)(qa - pa)) & ~bad;
  d = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, df), __builtin_bit_cast(short2v, df), d,
                             false);
  nacc += ~bad & 0x00010001u;
}

// A known pixel value v (0..255) in one half of a packed int16 pair, read as
// a binary16 bit pattern: the subnormal v * 2^-24, exactly.  Used as an FMA
// operand it becomes a mixed-precision FMA with no separate conversion.
static __device__ __forceinline__ float half_lo(uint32_t pp) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(pp & 0xffffu));
}
static __device__ __forceinline__ float half_hi(uint32_t pp) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(pp >> 16));
}

// ---------------------------------------------------------------- phases
// All functions below are called by every thread of the workgroup.

// Fixed tables, once per workgroup.  utab: the ring pixels of each footprint row taken left to
// right in pairs of horizontal neighbours (a lone pixel gets a dummy
// partner); lane fy owns footprint row fy, a wave scan orders the rows.
static __device__ __forceinline__ void phase_tables(const DevParams& p, const MainLds& L,
                                                    BlockShared& sh) {
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int B = p.B, r = p.r, W = p.W, Wd = p.Wd, F = p.F;
  for (int k = tid; k < 2 * Wd; k += kThreads) L.rowbits[k] = 0ull;
  if (wave == 0) {
    const int fy = lane;
    const bool full = fy < r || fy >= r + B;
    int cnt = 0;
    if (fy < F) cnt = full ? (F + 1) / 2 : 2 * ((r + 1) / 2);
    const int x = wave_incl_scan(cnt);
    int pos = x - cnt;
    if (fy < F) {
      if (full) {
        for (int c = 0; c < F; c += 2)
          L.utab[pos++] = (uint32_t)(fy * p.Wp + c) | ((uint32_t)(c + 1 >= F) << 16);
      } else {
        for (int c = 0; c < r; c += 2)
          L.utab[pos++] = (uint32_t)(fy * p.Wp + c) | ((uint32_t)(c + 1 >= r) << 16);
        for (int c = r + B; c < F; c += 2)
          L.utab[pos++] = (uint32_t)(fy * p.Wp + c) | ((uint32_t)(c + 1 >= F) << 16);
      }
    }
    if (lane == 63) sh.NU = x;
  }
  __syncthreads();
}

// Stage the window of the block whose window origin is (ox, oy).  A lane
// owns a segment of four window columns of one row (S = ceil(Wd / 4)
// segments a row, 64 / S rows per wave and pass) and reads the five values
// it needs (its four pixels and the right partner of the last) with one
// 12-byte load from the dword-aligned element below; a funnel shift aligns
// them.  Pixels outside the frame or past the window's last column become
// unknown (-1).  Reads stay within the value plane and its guard bands: a
// segment with an in-frame pixel starts at most 6 elements before the plane
// or ends at most 5 after it, and segments entirely outside (masked anyway)
// are clamped into the same range.  Each lane also ORs the availability bits
// of its four pixels into the row's 128-bit mask (rowbits, cleared by
// phase_tables).  stage_issue starts the loads, stage_finish writes LDS and
// ends with a barrier; phase_stage does both.
constexpr int kStagePass = 6;     // window rows a wave loads per lane row group at once

// The first kStagePass passes of a lane's window loads, held in registers so
// that the kernel can issue them before unrelated latency-bound work.
struct StageRegs {
  uint32_t w0[kStagePass], w1[kStagePass], w2[kStagePass], sh[kStagePass];
};

struct StageGeom {
  int S, R, g, c0, gx, rstep, npx;
  uint32_t colbad;
};

static __device__ __forceinline__ StageGeom stage_geom(const DevParams& p, int ox) {
  StageGeom G;
  const int lane = lane_id();
  G.S = (p.Wd + 3) >> 2;
  G.R = 64 / G.S;
  G.g = lane / G.S;
  G.c0 = 4 * (lane - G.g * G.S);
  G.gx = ox + G.c0;
  G.rstep = G.R * (kThreads / 64);
  G.npx = p.width * p.height;
  // unknown marks of the five values from the column tests alone (bit q)
  G.colbad = 0;
#pragma unroll
  for (int q = 0; q < 5; ++q)
    G.colbad |= (uint32_t)((unsigned)(G.gx + q) >= (unsigned)p.width || G.c0 + q >= p.Wd) << q;
  return G;
}

static __device__ __forceinline__ void stage_load(const FrameArgs& a, const DevParams& p,
                                                  const StageGeom& G, int oy, int wy0,
                                                  StageRegs& S) {
#pragma unroll
  for (int t = 0; t < kStagePass; ++t) {
    const int wy = wy0 + t * G.rstep;
    const int gy = oy + wy;
    const int cy = min(max(gy, 0), p.height - 1);
    const int e = cy * p.width + G.gx;
    const int e2 = min(max(e & ~1, -kValGuard), G.npx + 2);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.val + e2);
    S.sh[t] = (uint32_t)(e & 1) << 4;
    S.w0[t] = src[0]; S.w1[t] = src[1]; S.w2[t] = src[2];
  }
}

static __device__ __forceinline__ void stage_store(const DevParams& p, const MainLds& L,
                                                   const StageGeom& G, int oy, int wy0,
                                                   const StageRegs& S) {
  const int Wd = p.Wd;
#pragma unroll
  for (int t = 0; t < kStagePass; ++t) {
    const int wy = wy0 + t * G.rstep;
    if (G.g >= G.R || wy >= Wd) continue;
    const int gy = oy + wy;
    const uint32_t bad = (gy >= 0 && gy < p.height) ? G.colbad : 0x1fu;
    // x0 = (p0, p1), x1 = (p2, p3), low half of x2 = p4
    const uint32_t x0 = __builtin_amdgcn_alignbit(S.w1[t], S.w0[t], S.sh[t]);
    const uint32_t x1 = __builtin_amdgcn_alignbit(S.w2[t], S.w1[t], S.sh[t]);
    const uint32_t x2 = S.w2[t] >> S.sh[t];
    uint32_t pr[4] = {x0, __builtin_amdgcn_alignbit(x1, x0, 16), x1,
                      __builtin_amdgcn_alignbit(x2, x1, 16)};
#pragma unroll
    for (int q = 0; q < 4; ++q)
      pr[q] |= (((bad >> q) & 1u) ? 0x0000ffffu : 0u) | (((bad >> (q + 1)) & 1u) ? 0xffff0000u : 0u);
    // availability bits of the row: this segment's nibble (rows cleared by
    // phase_tables)
    uint32_t nib = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) nib |= (uint32_t)((pr[q] & 0x8000u) == 0u) << q;
    if (nib)
      atomicOr(reinterpret_cast<uint32_t*>(L.rowbits) + 4 * wy + (G.c0 >> 5), nib << (G.c0 & 31));
    uint32_t* dst = L.winp + wy * p.Wp + G.c0;
    if ((Wd & 3) == 0 && (p.Wp & 3) == 0) {
      *reinterpret_cast<uint4*>(dst) = make_uint4(pr[0], pr[1], pr[2], pr[3]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (G.c0 + q < Wd) dst[q] = pr[q];
    }
  }
}

// Loads of the first passes (issued early by the caller) are in S; the rest
// of the window, if any, is loaded and stored here.  Ends with a barrier.
static __device__ __forceinline__ void stage_finish(const FrameArgs& a, const DevParams& p,
                                                    const MainLds& L, const StageGeom& G, int oy,
                                                    const StageRegs& S) {
  const int wave = wave_id();
  int wy0 = wave * G.R + G.g;
  stage_store(p, L, G, oy, wy0, S);
  for (wy0 += kStagePass * G.rstep; wy0 < p.Wd + G.g; wy0 += kStagePass * G.rstep) {
    StageRegs T;
    stage_load(a, p, G, oy, wy0, T);
    stage_store(p, L, G, oy, wy0, T);
  }
  __syncthreads();
}

static __device__ __forceinline__ void stage_issue(const FrameArgs& a, const DevParams& p,
                                                   const StageGeom& G, int oy, StageRegs& S) {
  stage_load(a, p, G, oy, wave_id() * G.R + G.g, S);
}

static __device__ __forceinline__ void phase_stage(const FrameArgs& a, const DevParams& p,
                                                   const MainLds& L, int ox, int oy) {
  const StageGeom G = stage_geom(p, ox);
  StageRegs S;
  stage_issue(a, p, G, oy, S);
  stage_finish(a, p, L, G, oy, S);
}

struct RingStats { int n0, phi, sum; };

// Context units of the block (footprint origin qbase in the window) and ring
// statistics; horizontal B-runs of every window row by doubling.  Ends with a
// barrier.
// NUe >= NU: units NU .. NUe - 1 are the block's own positions in pairs of
// columns (B x B / 2 of them, for a block that holds received pixels; the
// lost ones read -1 and drop out of every sum).
static __device__ __forceinline__ RingStats phase_context(const DevParams& p, const MainLds& L,
                                                          BlockShared& sh, int NU, int NUe) {
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int qbase = p.W * p.Wp + p.W;
  {
    int c = 0, vmin = 255, vmax = 0, vsum = 0;
    for (int u = tid; u < NUe; u += kThreads) {
      int off;
      uint32_t qp;
      if (u < NU) {
        const uint32_t e = L.utab[u];
        off = (int)(e & 0xffffu);
        qp = L.winp[qbase + off];
        if (e >> 16) qp |= 0xffff0000u;
      } else {
        const int k2 = 2 * (u - NU), iy = k2 / p.B, ix = k2 - iy * p.B;
        off = (p.r + iy) * p.Wp + p.r + ix;
        qp = L.winp[qbase + off];
      }
      L.qu[u] = make_uint2(qp, (uint32_t)off);
      const int va = (int)(int16_t)(qp & 0xffffu), vb = (int)(int16_t)(qp >> 16);
      if (va >= 0) { ++c; vmin = min(vmin, va); vmax = max(vmax, va); vsum += va; }
      if (vb >= 0) { ++c; vmin = min(vmin, vb); vmax = max(vmax, vb); vsum += vb; }
    }
    for (int u = NUe + tid; u < align32(NUe); u += kThreads) L.qu[u] = make_uint2(0xffffffffu, 0u);
    c = wave_sum(c); vmin = wave_min(vmin); vmax = wave_max(vmax); vsum = wave_sum(vsum);
    if (lane == 0) {
      sh.red_i[wave][0] = c; sh.red_i[wave][1] = vmin;
      sh.red_i[wave][2] = vmax; sh.red_i[wave][3] = vsum;
    }
  }
  for (int row = tid; row < p.Wd; row += kThreads) {
    uint64_t lo = L.rowbits[2 * row], hi = L.rowbits[2 * row + 1];
    for (int s = 1; s < p.B; s <<= 1) {           // B is a power of two
      uint64_t tlo, thi;
      shr128(lo, hi, s, tlo, thi);
      lo &= tlo; hi &= thi;
    }
    L.runbits[2 * row] = lo; L.runbits[2 * row + 1] = hi;
  }
  __syncthreads();
  RingStats rs;
  int n0 = 0, vmin = 255, vmax = 0, vsum = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    n0 += sh.red_i[w][0]; vmin = min(vmin, sh.red_i[w][1]);
    vmax = max(vmax, sh.red_i[w][2]); vsum += sh.red_i[w][3];
  }
  rs.n0 = n0;
  rs.phi = n0 > 0 ? vmax - vmin : 0;
  rs.sum = vsum;
  return rs;
}

// Admissible prototypes: vertical AND of B runs per displacement row shifted
// to displacement columns (cmask), row counts and prefix, then the candidate
// list in raster order (candidate words, see cand_off).
// Also resets the per-bucket maxima and counts.  Returns M; ends with a
// barrier.
static __device__ __forceinline__ int phase_candidates(const DevParams& p, const MainLds& L,
                                                       BlockShared& sh) {
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int B = p.B, r = p.r, W = p.W, Wp = p.Wp, D2 = 2 * W + 1, nw = kThreads / 64;
  int rowcnt = 0;
  uint64_t mlo = 0ull, mhi = 0ull;
  if (tid < D2) {
    uint64_t lo = ~0ull, hi = ~0ull;
    for (int k = 0; k < B; ++k) { lo &= L.runbits[2 * (r + tid + k)]; hi &= L.runbits[2 * (r + tid + k) + 1]; }
    shr128(lo, hi, r, mlo, mhi);
    if (D2 < 64) { mlo &= (1ull << D2) - 1ull; mhi = 0; }
    else { mhi &= (D2 >= 128) ? ~0ull : ((1ull << (D2 - 64)) - 1ull); }
    // prototypes never overlap the block: displacements with |dy| < B and
    // |dx| < B are out (for a fully lost block they are unavailable anyway)
    if (abs(tid - W) < B) {
      const int c0 = max(0, W - B + 1), c1 = min(D2 - 1, W + B - 1);
      uint64_t klo, khi;                      // bits c0 .. c1
      shr128(~0ull, ~0ull, 127 - (c1 - c0), klo, khi);
      if (c0 >= 64) { khi = klo << (c0 - 64); klo = 0ull; }
      else if (c0 > 0) { khi = (khi << c0) | (klo >> (64 - c0)); klo <<= c0; }
      mlo &= ~klo; mhi &= ~khi;
    }
    L.cmask[2 * tid] = mlo; L.cmask[2 * tid + 1] = mhi;
    rowcnt = __popcll(mlo) + __popcll(mhi);
  }
  if (D2 <= 64) {                        // every row in wave 0
    if (wave == 0) {
      const int incl = wave_incl_scan(rowcnt);
      if (lane < D2) sh.rowbase[lane] = incl - rowcnt;
      if (lane == 63) sh.M = incl;
    }
  } else {
    int tot = 0;
    const int rb = block_excl_scan(rowcnt, sh.scan, &tot);   // barriers inside
    if (tid < D2) sh.rowbase[tid] = rb;
    if (tid == 0) sh.M = tot;
  }
  if (tid < p.nrad) { sh.bmax[tid] = 0xFFF0000000000000ull; sh.bcnt[tid] = 0; }
  __syncthreads();
  const unsigned long long lut0 = p.bucket_lut[0], lut1 = p.bucket_lut[1], lut2 = p.bucket_lut[2];
  if (D2 <= 64) {
    // one 64-bit mask per displacement row; thread t takes (row, group of 8
    // columns) units t, t + 256, ...: the rank of the group's first column is
    // the row offset plus the set bits below it, then its set bits in order
    const int ngr = (D2 + 7) >> 3;
    const int nunits = D2 * ngr;
    const float inv_ngr = 1.0f / (float)ngr;
    for (int u = tid; u < nunits; u += kThreads) {
      int dyi = (int)(((float)u + 0.5f) * inv_ngr);          // u / ngr (u < 2^12: exact)
      dyi -= dyi * ngr > u ? 1 : 0;
      dyi += (dyi + 1) * ngr <= u ? 1 : 0;
      const int g = u - dyi * ngr;
      const uint64_t m = L.cmask[2 * dyi];
      uint32_t bits = (uint32_t)(m >> (8 * g)) & 0xffu;
      if (!bits) continue;
      int pos = sh.rowbase[dyi] + __popcll(m & ((1ull << (8 * g)) - 1ull));
      const int ady = abs(dyi - W);
      while (bits) {
        const int dxi = 8 * g + __ffs(bits) - 1;
        bits &= bits - 1u;
        const int rho = max(ady, abs(dxi - W));
        const uint32_t bk = (uint32_t)((rho < 16 ? lut0 : lut1) >> (4 * (rho & 15))) & 15u;
        L.cand[pos++] = (uint32_t)(dyi * Wp + dxi) | (bk << 14);
      }
    }
  } else {
    // wave w writes displacement rows w, w + 4, ..., lanes along the columns;
    // the masks and offsets of kAhead rows are read before any row is written
    constexpr int kAhead = 5;
    for (int dy0 = wave; dy0 < D2; dy0 += kAhead * nw) {
      uint64_t ml[kAhead], mh[kAhead];
      int rbv[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int dyi = min(dy0 + u * nw, D2 - 1);
        ml[u] = L.cmask[2 * dyi];
        mh[u] = L.cmask[2 * dyi + 1];
        rbv[u] = sh.rowbase[dyi];
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int dyi = dy0 + u * nw;
        if (dyi >= D2) break;
        const int ady = abs(dyi - W);
        for (int dxi = lane; dxi < D2; dxi += 64) {
          const bool ok = dxi < 64 ? ((ml[u] >> dxi) & 1ull) : ((mh[u] >> (dxi - 64)) & 1ull);
          if (ok) {
            const int rank = dxi < 64 ? __popcll(ml[u] & ((1ull << dxi) - 1ull))
                                      : __popcll(ml[u]) + __popcll(mh[u] & ((1ull << (dxi - 64)) - 1ull));
            const int rho = max(ady, abs(dxi - W));
            const unsigned long long lw = rho < 16 ? lut0 : (rho < 32 ? lut1 : lut2);
            const uint32_t bk = (uint32_t)(lw >> (4 * (rho & 15))) & 15u;
            L.cand[rbv[u] + rank] = (uint32_t)(dyi * Wp + dxi) | (bk << 14);
          }
        }
      }
    }
  }
  __syncthreads();
  return sh.M;
}

// Exact integer distance of the candidate whose footprint origin is `base`
// in the window, over the ring pixels known in both rings, two pixels per
// step (packed int16 difference, masked, v_dot2).  Returns d and the count n.
static __device__ __forceinline__ void cand_distance(const MainLds& L, int base, int NU, int& d_out,
                                                     int& n_out) {
  int d = 0;
  uint32_t nacc = 0;
  int u = 0;
  for (; u + 8 <= NU; u += 8) {
    uint2 qq[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) qq[t] = L.qu[u + t];
#pragma unroll
    for (int t = 0; t < 8; ++t) pair_dist(qq[t].x, L.winp[base + (int)qq[t].y], d, nacc);
  }
  for (; u < NU; ++u) {
    const uint2 qq = L.qu[u];
    pair_dist(qq.x, L.winp[base + (int)qq.y], d, nacc);
  }
  d_out = d;
  n_out = (int)(nacc & 0xffffu) + (int)(nacc >> 16);
}

// Six-operation form of pair_dist: unknown halves of either side give a
// zero difference; `nbad` counts them (sdot2 of the 0 / -1 masks).
// The masking is one v_bfi_b32 (written as an ALU-only asm statement: the
// compiler otherwise turns the and-not of a sign mask into per-half compares
// and selects, five more instructions).
static __device__ __forceinline__ void pair_dist6(uint32_t q, uint32_t pp, int& d, int& nbad) {
  const short2v qa = __builtin_bit_cast(short2v, q), pa = __builtin_bit_cast(short2v, pp);
  const short2v bad = (qa | pa) >> (short2v){15, 15};          // -1 where unknown
  const uint32_t diff = __builtin_bit_cast(uint32_t, (short2v)(qa - pa));
  uint32_t dm;
  asm("v_bfi_b32 %0, %1, 0, %2" : "=v"(dm) : "v"(__builtin_bit_cast(uint32_t, bad)), "v"(diff));
  const short2v df = __builtin_bit_cast(short2v, dm);
  d = __builtin_amdgcn_sdot2(df, df, d, false);
  nbad = __builtin_amdgcn_sdot2(bad, bad, nbad, false);
}

// pair_dist6 for a context pair known in both halves: only the window side
// can be unknown, one operation fewer.
static __device__ __forceinline__ void pair_dist5(uint32_t q, uint32_t pp, int& d, int& nbad) {
  const short2v qa = __builtin_bit_cast(short2v, q), pa = __builtin_bit_cast(short2v, pp);
  const short2v bad = pa >> (short2v){15, 15};                 // -1 where unknown
  const uint32_t diff = __builtin_bit_cast(uint32_t, (short2v)(qa - pa));
  uint32_t dm;
  asm("v_bfi_b32 %0, %1, 0, %2" : "=v"(dm) : "v"(__builtin_bit_cast(uint32_t, bad)), "v"(diff));
  const short2v df = __builtin_bit_cast(short2v, dm);
  d = __builtin_amdgcn_sdot2(df, df, d, false);
  nbad = __builtin_amdgcn_sdot2(bad, bad, nbad, false);
}

// Distance of one candidate per lane (footprint origin `base`; a lane
// without a candidate passes 0 and ignores the result).  Every lane reads
// the same unit (q pair, offset) -- an LDS broadcast -- and its own window
// pair; 16 units per step keep 32 independent reads in flight.  NU32 is a
// multiple of 32 (padded units are unknown pairs).
static __device__ __forceinline__ void cand_distance_wave(const MainLds& L, int base, int NU32,
                                                          int& d_out, int& n_out) {
  int d = 0, nbad = 0;
  for (int u0 = 0; u0 < NU32; u0 += 16) {
    uint2 qq[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) qq[t] = L.qu[u0 + t];
    uint32_t pv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) pv[t] = L.winp[base + (int)qq[t].y];
#pragma unroll
    for (int t = 0; t < 16; ++t) pair_dist6(qq[t].x, pv[t], d, nbad);
  }
  d_out = d;
  n_out = 2 * NU32 - nbad;
}

// Context units of a geometry fixed at compile time (block B, ring R,
// search radius W): the same enumeration as phase_tables (footprint rows top
// to bottom; full rows in pairs of columns, the rows beside the block in the
// left and right ring parts), so unit u of the table matches qu[u].
template <int B, int R, int W>
struct FixedGeom {
  static constexpr int kB = B, kR = R, kW = W;
  static constexpr int F = B + 2 * R;
  static constexpr int Wd = B + 2 * R + 2 * W;
  static constexpr int Wp = Wd | 1;   // LDS row pitch, as DevParams::Wp
  static constexpr int NU = 2 * R * ((F + 1) / 2) + B * 2 * ((R + 1) / 2);
  static_assert(F % 2 == 0 && R % 2 == 0, "units must be whole pixel pairs");
  static_assert(NU % 32 == 0, "unit count must fill the 16-unit steps without padding");
  struct Table { int off[NU]; };
  static constexpr Table table() {
    Table t{};
    int u = 0;
    for (int fy = 0; fy < F; ++fy) {
      const bool full = fy < R || fy >= R + B;
      for (int c = 0; c < F; c += 2)
        if (full || c < R || c >= R + B) t.off[u++] = fy * Wp + c;
    }
    return t;
  }
  static constexpr Table kUnits = table();
};

// cand_distance_wave for a fixed geometry: the window offset of every unit
// is a compile-time constant, so each lane's window reads are immediate
// offsets from its own footprint origin and do not wait for the unit table.
// QKnown: every context pixel of the block is known (pair_dist5).
template <class G, bool QKnown>
static __device__ __forceinline__ void cand_distance_fixed(const MainLds& L, int base, int& d_out,
                                                           int& n_out) {
  int d = 0, nbad = 0;
  const uint32_t* wb = L.winp + base;
  // The context pairs are the same for every lane: lane t holds those of
  // units t, t + 64, ... in registers and v_readlane hands each to the
  // whole wave, so that the only LDS read per unit is the lane's own window
  // pair.  Two 16-unit steps in flight: the window reads of step k + 1 are
  // issued before the arithmetic of step k; scheduling barriers keep the
  // compiler from hoisting further reads (registers)
  constexpr int kSteps = G::NU / 16;
  constexpr int kQ = (G::NU + 63) / 64;
  const int lane = lane_id();
  uint32_t qreg[kQ];
#pragma unroll
  for (int c = 0; c < kQ; ++c) qreg[c] = 64 * c + lane < G::NU ? L.qu[64 * c + lane].x : 0u;
  uint32_t pv[2][16];
#pragma unroll
  for (int t = 0; t < 16; ++t) pv[0][t] = wb[G::kUnits.off[t]];
#pragma unroll
  for (int k = 0; k < kSteps; ++k) {
    if (k + 1 < kSteps) {
#pragma unroll
      for (int t = 0; t < 16; ++t) pv[(k + 1) & 1][t] = wb[G::kUnits.off[16 * (k + 1) + t]];
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int u = 16 * k + t;
      const uint32_t q = (uint32_t)__builtin_amdgcn_readlane((int)qreg[u / 64], u % 64);
      if (QKnown) pair_dist5(q, pv[k & 1][t], d, nbad);
      else pair_dist6(q, pv[k & 1][t], d, nbad);
    }
    // pin the sums here: otherwise the (pure) dot products sink past the
    // loop and every masked difference stays live until the end
    asm volatile("" : "+v"(d), "+v"(nbad));
    __builtin_amdgcn_sched_barrier(0);
  }
  d_out = d;
  n_out = 2 * G::NU - nbad;
}

using Geom16 = FixedGeom<16, 4, 24>;

}  // namespace skm
