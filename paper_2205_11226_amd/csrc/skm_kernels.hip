// gfx950 kernels of block-mode scalable K-MMSE concealment.
//
// One lost block is processed by one workgroup of 4 wave64.  Its whole search
// window (B + 2r + 2W pixels a side) is staged once in LDS from coalesced
// row reads of the frame; every later step (context gather, prototype
// admissibility, distances, weights, weighted average) reads LDS only.
//
// Paper references (Koloda et al., arXiv 2205.11226):
//   context mean / flatness        Sec. "Basic reconstruction layer", eq. mean;
//                                  Sec. "Layer switching" (phi)
//   kernel weights, IDL estimate   eq. weights, eq. slpe (H_YY = sigma^2 N_y I)
//   normalisation factor nu        eq. factor (raw weight sum, negative exponent)
//   support-area expansion         Sec. "Intermediate dynamic layer"
//   profile gate                   Sec. "SK-MMSE profiles"
//   transfer of estimates into S   end of Sec. "K-MMSE overview"
#include <math.h>

#include <type_traits>

#include "skm_device.h"

namespace skm {

// ---------------------------------------------------------- state / setup

// Host-visible copy of the frame state (pinned, coherent host memory): the
// host reads it after synchronizing the stream instead of a copy node.
__device__ __forceinline__ void publish_state_to(const RoundState* st, RoundState* h) {
  if (!h) return;
  h->n_lost = st->n_lost; h->remaining = st->remaining; h->round = st->round;
  h->err = st->err; h->n_hql = st->n_hql;
  h->n_avail = st->n_avail; h->sum_avail = st->sum_avail;
}
__device__ __forceinline__ void publish_state(const FrameArgs& a) {
  publish_state_to(a.st, a.hstate);
}

// Loss geometry, one pass over the frame.  Grid (ceil(width/1024), bands of
// B rows); each thread owns four adjacent columns of a band (32-bit loads and
// stores where the rows allow them): copies received pixels to `work` (lost
// ones become 128 and are never read), writes the value plane (-1 = lost),
// and the B / 4 threads of one cell (for B = 2: each thread's two cells) vote
// whether the cell holds a lost pixel.  A lost pixel outside the full-cell
// grid is an error.
// Lost cells are ORed into a bit table with device-scope atomics (coherent
// across XCDs without a cache flush); the workgroup that finishes last lists
// them in raster order, clears the table and starts the frame state.
// Workgroup (wgx, band) of a frame whose geometry pass has nwg workgroups;
// returns true in the workgroup that finished the frame (it listed the cells).
static __device__ bool init_body(const FrameArgs& a, const DevParams& p, int wgx, int band,
                                 unsigned nwg) {
  __shared__ int s_scan[kThreads / 64];
  __shared__ int s_last;
  const int lane = lane_id(), wave = wave_id(), tid = threadIdx.x;
  const int x = (wgx * kThreads + tid) * 4;
  const int B = p.B;
  const int y0 = band * B;
  const int rows = min(B, p.height - y0);
  RoundState* st = a.st;
  // 32-bit accesses when the four columns are in the frame and aligned
  const bool vec = x + 3 < p.width && ((p.stride | p.width) & 3) == 0 &&
                   (((uintptr_t)a.frame | (uintptr_t)a.mask | (uintptr_t)a.work) & 3) == 0;
  int nl = 0, nl_hi = 0;                             // lost pixels; of columns 2, 3
  if (vec) {
    uint32_t mk[kMaxB], fv[kMaxB];
#pragma unroll
    for (int i = 0; i < kMaxB; ++i) {
      const size_t off = (size_t)(y0 + min(i, rows - 1)) * p.stride + x;
      mk[i] = *reinterpret_cast<const uint32_t*>(a.mask + off);
      fv[i] = *reinterpret_cast<const uint32_t*>(a.frame + off);
    }
#pragma unroll
    for (int i = 0; i < kMaxB; ++i) {
      if (i < rows) {
        uint32_t wk = 0, v01 = 0, v23 = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool lost = ((mk[i] >> (8 * q)) & 0xffu) != 0u;
          const uint32_t pix = (fv[i] >> (8 * q)) & 0xffu;
          wk |= (lost ? 128u : pix) << (8 * q);
          const uint32_t vv = lost ? 0xffffu : pix;
          if (q < 2) v01 |= vv << (16 * q); else v23 |= vv << (16 * (q - 2));
          nl += lost;
          nl_hi += q >= 2 && lost;
        }
        const int y = y0 + i;
        *reinterpret_cast<uint32_t*>(a.work + (size_t)y * p.stride + x) = wk;
        *reinterpret_cast<uint2*>(a.val + (size_t)y * p.width + x) = make_uint2(v01, v23);
      }
    }
  } else {
    for (int q = 0; q < 4; ++q) {
      const int xq = x + q;
      if (xq >= p.width) break;
      for (int i = 0; i < rows; ++i) {
        const int y = y0 + i;
        const size_t off = (size_t)y * p.stride + xq;
        const bool lost = a.mask[off] != 0;
        const uint8_t v = a.frame[off];
        a.work[off] = lost ? (uint8_t)128 : v;
        a.val[(size_t)y * p.width + xq] = lost ? (int16_t)-1 : (int16_t)v;
        nl += lost;
        nl_hi += q >= 2 && lost;
      }
    }
  }
  uint64_t lm = 0, lm_hi = 0;
  bool any_bad;
  if (B == 2) {
    // two cells per thread: columns 0-1 and 2-3
    const int cx = x >> 1;
    const bool in0 = band < p.gh && cx < p.gw, in1 = band < p.gh && cx + 1 < p.gw;
    const int n0 = nl - nl_hi;
    lm = __ballot(in0 && n0 > 0);
    lm_hi = __ballot(in1 && nl_hi > 0);
    any_bad = __ballot((n0 > 0 && !in0) || (nl_hi > 0 && !in1)) != 0ull;
  } else {
    const int TB = B >> 2;                           // threads per cell
    const bool in_cells = band < p.gh && x < p.gw * B;
    int v = nl;
    for (int o = 1; o < TB; o <<= 1) v += __shfl_xor(v, o, 64);   // cells never straddle waves
    const bool leader = in_cells && (lane & (TB - 1)) == 0;
    // a cell with any lost pixel is a block (its received pixels join the context)
    const uint64_t lv = __ballot(leader && v > 0);
    for (int k = 0; k < 64 / TB; ++k) lm |= ((lv >> (k * TB)) & 1ull) << k;
    any_bad = __ballot(nl > 0 && !in_cells) != 0ull;
  }
  if (lane == 0) {
    unsigned int sink = 0;
    if (lm | lm_hi) {
      // this wave's cells are consecutive from cell cb: 256 / B of them, bit
      // k of the 128-bit run (lo, hi) for cell cb + k
      const int cb = band * p.gw + (wgx * kThreads + wave * 64) * 4 / B;
      uint64_t lo = lm, hi = 0;
      if (B == 2) {
        lo = 0;
        for (int k = 0; k < 32; ++k) {
          lo |= ((lm >> k) & 1ull) << (2 * k) | ((lm_hi >> k) & 1ull) << (2 * k + 1);
          hi |= ((lm >> (k + 32)) & 1ull) << (2 * k) | ((lm_hi >> (k + 32)) & 1ull) << (2 * k + 1);
        }
      }
      const uint32_t src[4] = {(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
      const int w = cb >> 5, sh = cb & 31;
      for (int k = 0; k < 5; ++k) {
        uint32_t pk = k < 4 ? src[k] << sh : 0u;
        if (k > 0 && sh) pk |= src[k - 1] >> (32 - sh);
        if (pk) sink ^= atomicOr(&a.cellbits[w + k], pk);
      }
    }
    if (any_bad) sink ^= (unsigned int)atomicOr(&st->err_geo, kErrPartial);
    asm volatile("" ::"v"(sink));        // the atomics have completed before the ticket
  }
  __syncthreads();
  if (tid == 0) {
    const unsigned t = atomicAdd(&st->ticket, 1u);
    s_last = t + 1 == nwg;
    if (s_last) atomicExch(&st->ticket, 0u);
  }
  __syncthreads();
  if (!s_last) return false;

  // ordered compaction: thread t takes a contiguous run of table words
  const int ncell = p.gh * p.gw, nw = (ncell + 31) >> 5;
  const int per = (nw + kThreads - 1) / kThreads;
  const int w0 = min(nw, tid * per), w1 = min(nw, w0 + per);
  // eight independent loads in flight per step (a large table, e.g. 2 x 2
  // cells, gives each thread tens of words)
  int n = 0;
  for (int w = w0; w < w1; w += 8) {
    uint32_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      v[q] = w + q < w1 ? __hip_atomic_load(&a.cellbits[w + q], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) n += __popc(v[q]);
  }
  int tot = 0;
  int pos = block_excl_scan(n, s_scan, &tot);
  for (int w = w0; w < w1; w += 8) {
    uint32_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      v[q] = w + q < w1 ? __hip_atomic_load(&a.cellbits[w + q], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      uint32_t bits = v[q];
      while (bits) {
        const int b = __ffs(bits) - 1;
        bits &= bits - 1u;
        a.blk[pos] = (w + q) * 32 + b;
        a.bstate[pos] = 0;
        ++pos;
      }
      if (w + q < w1)
        __hip_atomic_store(&a.cellbits[w + q], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (tid == 0) {
    st->n_lost = tot; st->remaining = tot; st->round = 1;
    st->err = atomicExch(&st->err_geo, 0);
    st->n_hql = 0; st->n_avail = 0; st->sum_avail = 0;
    st->ctx_nq = 0; st->ctx_max = 0;
    publish_state(a);
  }
  return true;
}

__global__ __launch_bounds__(kThreads) void k_init(FrameArgs a, DevParams p) {
  init_body(a, p, blockIdx.x, blockIdx.y, gridDim.x * gridDim.y);
}

// ------------------------------------------------------------- round prep
// One wave per pending block: |m0| = known in-frame context pixels, with their
// sum, minimum and maximum (the context mean and flatness of the BRL gate).
// Each workgroup adds its (blocks with |m0| >= r B, largest |m0|) to the
// round state's context rule (integer atomics, so the result is order-free).
// One wave: context statistics of pending block i over its footprint (the
// ring and the block's own received pixels; lost ones read -1), written to
// m0cnt / ring; lane 0 adds the block to (nq, mx).
static __device__ __forceinline__ void prep_one(const FrameArgs& a, const DevParams& p, int i,
                                                int lane, int& my_nq, int& my_mx) {
  const int F = p.F, B = p.B, r = p.r;
  const int cell = a.blk[i];
  const int by = cell / p.gw, bx = cell - by * p.gw;
  const int xr = bx * B - r, yr = by * B - r;
  int c = 0, sum = 0, vmin = 255, vmax = 0;
  bool own = false;
#pragma unroll
  for (int fy0 = 0; fy0 < 2 * kMaxB; fy0 += 2) {     // two footprint rows per step, F <= 32
    const int fy = fy0 + (lane >> 5), fx = lane & 31;
    const int gy = yr + fy, gx = xr + fx;
    const bool use = fy < F && fx < F && gy >= 0 && gy < p.height && gx >= 0 && gx < p.width;
    const int cy = min(max(gy, 0), p.height - 1), cx = min(max(gx, 0), p.width - 1);
    const int v = a.val[(size_t)cy * p.width + cx];
    if (use && v >= 0) {
      ++c; sum += v; vmin = min(vmin, v); vmax = max(vmax, v);
      own = own || (fy >= r && fy < r + B && fx >= r && fx < r + B);
    }
  }
  c = wave_sum(c);
  sum = wave_sum(sum);
  vmin = wave_min(vmin);
  vmax = wave_max(vmax);
  const bool partial = __ballot(own) != 0ull;
  if (lane == 0) {
    a.m0cnt[i] = c | (partial ? kPartialBit : 0);
    a.ring[i] = make_int2(sum, vmin | (vmax << 16));
    my_nq += c >= r * B;
    my_mx = max(my_mx, c);
  }
}

// Adds the per-wave (nq, mx) of a workgroup to the context rule of state st
// (one call per workgroup; every thread of the workgroup calls it).
static __device__ __forceinline__ void flush_context_rule(RoundState* st, int my_nq, int my_mx,
                                                          int (*s_nq), int (*s_mx)) {
  const int lane = lane_id(), wave = wave_id();
  if (lane == 0) { s_nq[wave] = my_nq; s_mx[wave] = my_mx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nq = 0, mx = 0;
    for (int w = 0; w < kThreads / 64; ++w) { nq += s_nq[w]; mx = max(mx, s_mx[w]); }
    note_context_rule(st, nq, mx);
  }
  __syncthreads();
}

// One wave per pending block: |m0| = known in-frame context pixels, with their
// sum, minimum and maximum (the context mean and flatness of the BRL gate).
// Each workgroup adds its (blocks with |m0| >= r B, largest |m0|) to the
// round state's context rule (integer atomics, so the result is order-free).
__global__ __launch_bounds__(kThreads) void k_round_prep(FrameArgs a, DevParams p) {
  __shared__ int s_nq[kThreads / 64], s_mx[kThreads / 64];
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) st->n_hql = 0;
  const int n_lost = st->n_lost;
  const int lane = lane_id(), wave = wave_id();
  int my_nq = 0, my_mx = 0;
  // with a grid of whole XCD groups, XCD x takes the x-th contiguous eighth
  // of the blocks, as in the estimation kernel (its L2 then holds the rings)
  constexpr int nwv = kThreads / 64;
  int i0 = blockIdx.x * nwv + wave, i1 = n_lost, step = gridDim.x * nwv;
  if ((gridDim.x & 7) == 0) {
    const int per8 = (n_lost + 7) >> 3, xcd = blockIdx.x & 7;
    i0 = xcd * per8 + (int)(blockIdx.x >> 3) * nwv + wave;
    i1 = min(n_lost, (xcd + 1) * per8);
    step = (int)(gridDim.x >> 3) * nwv;
  }
  for (int i = i0; i < i1; i += step) {
    if (a.bstate[i] != 0) continue;
    prep_one(a, p, i, lane, my_nq, my_mx);
  }
  flush_context_rule(st, my_nq, my_mx, s_nq, s_mx);
}

// ----------------------------------------------------------- main kernel

size_t main_lds_bytes(const DevParams& p) {
  size_t offs[6];
  return est_lds_layout(p, offs);
}

__device__ void write_info(const FrameArgs& a, int i, int bx, int by, int layer, int round,
                           int n_cand, int n_complete, int radius, int flags, int phi,
                           int n0, double lnu) {
  if (!a.info || i >= a.cap) return;
  skm_block_info inf;
  inf.bx = bx; inf.by = by; inf.layer = layer; inf.round = round;
  inf.n_cand = n_cand; inf.n_complete = n_complete; inf.radius = radius;
  inf.flags = flags; inf.phi = phi; inf.n_ctx = n0; inf.log_nu = lnu;
  a.info[i] = inf;
}

__device__ void write_const_block(const FrameArgs& a, const DevParams& p, int i, int x0, int y0,
                                  double v, bool partial) {
  const int B2 = p.B * p.B;
  const uint8_t u = (uint8_t)fmin(fmax(floor(v + 0.5), 0.0), 255.0);
  for (int pix = threadIdx.x; pix < B2; pix += kThreads) {
    const int py = pix / p.B, px = pix - py * p.B;
    // a block holding received pixels keeps them
    if (!partial || a.val[(size_t)(y0 + py) * p.width + x0 + px] < 0)
      a.work[(size_t)(y0 + py) * p.stride + x0 + px] = u;
    if (a.xhat && i < a.cap) a.xhat[(size_t)i * B2 + pix] = (float)v;
  }
}

// KP bounds the candidates of one thread's contiguous slice (ceil(MC / 256))
// and KR the expansion radii; launch_main picks the smallest instance that
// fits the geometry.
// FG selects the distance loop of the 16 x 16 block, ring 4, radius 24
// geometry (compile-time unit offsets); launch_main uses it only there.
// pend (batched kernels; nullptr otherwise) counts the blocks this call
// leaves pending: deferred by the round's context rule, or waiting for HQL.
template <int KP, int KR, bool FG>
static __device__ __forceinline__ void est_block(const FrameArgs& a, const DevParams& p, int i,
                                                 int round, int dist_only,
                                                 unsigned char* lds_raw, BlockShared& sh,
                                                 int* pend) {
  RoundState* st = a.st;
  // the block's values in one round trip, tested afterwards
  const int bst = a.bstate[i], cell = a.blk[i], m0w = a.m0cnt[i];
  const int2 rg = a.ring[i];
  const bool cnn = p.mode == SKM_MODE_CNN && p.cnn_active;
  const int gsel = (cnn && !dist_only) ? (int)a.gate[i] : -1;
  // context rule of the round (prep or gate workgroups)
  const int nq = st->ctx_nq, maxm0 = st->ctx_max;
  if (bst != 0) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int B = p.B, r = p.r, W = p.W, Wp = p.Wp, D2 = 2 * W + 1;
  const int B2 = B * B;
  const int by = cell / p.gw, bx = cell - by * p.gw;
  const int x0 = bx * B, y0 = by * B;
  if (!dist_only && nq == 0 && maxm0 == 0) {
    if (tid == 0) {
      atomicOr(&st->err, kErrNoContext);
      if (pend) atomicAdd(pend, 1);
    }
    return;
  }
  const int n0 = m0w & (kPartialBit - 1);
  const bool partial = (m0w & kPartialBit) != 0;      // the block holds received pixels
  if (!dist_only && !(nq > 0 ? (n0 >= p.r * p.B) : (n0 == maxm0))) {
    if (pend && tid == 0) atomicAdd(pend, 1);          // deferred to a later round
    return;
  }


  // 1. BRL gate on the prep kernel's ring statistics: context mean for every
  //    pixel of the block (profile rule, or the learned gate's choice in CNN
  //    mode), without staging the window
  const int phi = n0 > 0 ? (rg.y >> 16) - (rg.y & 0xffff) : 0;
  const double mean = n0 > 0 ? (double)rg.x / (double)n0 : 0.0;
  const int relaxed_flag = (!dist_only && nq == 0) ? SKM_FLAG_CTX_RELAXED : 0;
  const bool profile_rule = p.mode == SKM_MODE_PROFILE || (p.mode == SKM_MODE_CNN && !cnn);
  if (!dist_only && (p.mode == SKM_MODE_BRL || (profile_rule && (double)phi <= p.t_phi) ||
                     gsel == SKM_LAYER_BRL)) {
    write_const_block(a, p, i, x0, y0, mean, partial);
    if (tid == 0) {
      write_info(a, i, bx, by, SKM_LAYER_BRL, round, -1, -1, 0, relaxed_flag, phi, n0, NAN);
      a.bstate[i] = round;
    }
    return;
  }

  // 2. stage the search window in LDS; context ring (packed pairs); row
  //    B-runs.  The window loads go out only now, so that blocks deferred or
  //    concealed by BRL above read no window; they land while the tables
  //    are built.
  const StageGeom SG = stage_geom(p, x0 - r - W);
  StageRegs SR;
  stage_issue(a, p, SG, y0 - r - W, SR);
  const EstLds E = carve_est_lds(lds_raw, p);
  phase_tables(p, E.m, sh);
  const int NU = sh.NU;
  stage_finish(a, p, E.m, SG, y0 - r - W, SR);
  // context units: the ring, then the block's own pixel pairs if it holds
  // received pixels.  Every ring pixel known and no own units: the distance
  // step masks the window side only
  const int NUe = partial ? NU + p.B * p.B / 2 : NU;
  const bool qfull = phase_context(p, E.m, sh, NU, NUe).n0 == 2 * NU && !partial;

  // 3. admissible prototypes in raster order
  phase_candidates(p, E.m, sh);
  const int M = sh.M;

  // 4. exact integer distances over the ring pixels known in both rings, one
  //    candidate per lane; bucket maxima of the log raw weights by atomic
  //    minima of their (negative) bit patterns
  const int nmin = max(1, (p.min_pct * n0 + 99) / 100);
  const double two_s2 = 2.0 * p.sigma2;
  int nc = 0, ncomp = 0;
  const int NU32 = align32(NUe);
  // one copy of the loop per distance routine, chosen once per block:
  // compile-time unit offsets with or without the context-side mask, or the
  // unit table (other geometries, and blocks with own units)
  auto dist_loop = [&](auto kind) {
    for (int j0 = wave * 64; j0 < M; j0 += kThreads) {     // uniform per wave
      const int j = j0 + lane;
      const bool act = j < M;
      const uint32_t cj = act ? E.cand[j] : 0u;
      const int base = cand_off(cj);
      int d, n;
      if constexpr (decltype(kind)::value < 2)
        cand_distance_fixed<Geom16, decltype(kind)::value == 0>(E.m, base, d, n);
      else
        cand_distance_wave(E.m, base, NU32, d, n);
      if (!act) continue;
      const bool ok = n >= nmin;
      nc += ok;
      ncomp += ok && n == n0;
      if (dist_only) {
        const int t = (base / Wp) * D2 + (base % Wp);
        a.dist[(size_t)i * p.ND + t] = ok ? d : -1;
        a.cnt[(size_t)i * p.ND + t] = ok ? n : 0;
        continue;
      }
      E.cand[j] = cj | ((uint32_t)n << 18);
      E.dist[j] = ok ? (uint32_t)d : ~0u;
      if (ok) {
        const int b = cand_bucket(cj);
        const double e = -(double)d / ((double)n * two_s2);
        atomicMin(&sh.bmax[b], (unsigned long long)__double_as_longlong(e));
        atomicAdd(&sh.bcnt[b], 1);
      }
    }
  };
  if constexpr (FG) {
    if (!partial && qfull) dist_loop(std::integral_constant<int, 0>{});
    else if (!partial) dist_loop(std::integral_constant<int, 1>{});
    else dist_loop(std::integral_constant<int, 2>{});
  } else {
    dist_loop(std::integral_constant<int, 2>{});
  }
  if (dist_only) {
    // displacements without an admissible prototype (cmask is intact: the
    // distance step wrote no LDS)
    for (int t = tid; t < p.ND; t += kThreads) {
      const int dyi = t / D2, dxi = t - dyi * D2;
      const uint64_t w = dxi < 64 ? E.m.cmask[2 * dyi] : E.m.cmask[2 * dyi + 1];
      const bool adm = (w >> (dxi & 63)) & 1ull;
      if (!adm) { a.dist[(size_t)i * p.ND + t] = -1; a.cnt[(size_t)i * p.ND + t] = 0; }
    }
    return;
  }
  nc = wave_sum_full(nc);
  ncomp = wave_sum_full(ncomp);
  if (lane == 0) { sh.red_i[wave][0] = nc; sh.red_i[wave][1] = ncomp; }
  __syncthreads();

  // 5. log nu per expansion radius.  bm[b] is the maximum log raw weight of
  //    bucket b.  Thread t owns the contiguous slice [t per, t per + per) of
  //    the candidates; each kept candidate's term exp(ell - bm[b_j]) stays in
  //    registers for the weights and goes to a register accumulator of its
  //    bucket; wave sums in fixed order; wave 0 combines the buckets <= b by
  //    a prefix log-sum-exp across lanes.
  const int per = (M + kThreads - 1) / kThreads;
  const int js = min(M, tid * per);
  double t_r[KP];
  uint32_t c_r[KP];
  {
    double acc[KR];
#pragma unroll
    for (int b = 0; b < KR; ++b) acc[b] = 0.0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int j = js + k;
      t_r[k] = -1.0;
      c_r[k] = 0u;
      if (k < per && j < M) {
        const uint32_t d = E.dist[j];
        const uint32_t cj = E.cand[j];
        c_r[k] = cj;
        if (d != ~0u) {
          const int bj = cand_bucket(cj);
          const double t = exp(-(double)d / ((double)cand_n(cj) * two_s2) -
                               __longlong_as_double((long long)sh.bmax[bj]));
          t_r[k] = t;
#pragma unroll
          for (int b = 0; b < KR; ++b) acc[b] += (b == bj) ? t : 0.0;
        }
      }
    }
#pragma unroll
    for (int b = 0; b < KR; ++b) {
      if (b < p.nrad) {
        const double s = wave_sum_full(acc[b]);
        if (lane == 0) sh.ps[wave][b] = s;
      }
    }
  }
  __syncthreads();
  if (wave == 0) {
    // lane b: (m, cs) = (max, sum of exp(ell - max)) over buckets <= b, cc
    // their candidate count.
    const int b = lane;
    const double bm = b < p.nrad ? __longlong_as_double((long long)sh.bmax[b]) : -INFINITY;
    double m, cs;
    int cc;
    // at most 8 radii (every variant of that case sums in this same order,
    // so that they agree bit for bit)
    const bool r8 = KR <= 8 || p.nrad <= 8;
    double fpair = 0.0;   // r8: exp(bm[lane & 7] - m[lane >> 3]) for lane & 7 <= lane >> 3
    if (r8) {
      // lane (g, h) = (lane >> 3, lane & 7) holds bucket h's term of prefix g:
      // one exponential per lane, then sums over the eight lanes of a group
      const int g = lane >> 3, h = lane & 7;
      const bool on = g < p.nrad && h <= g;
      const double bmh = on ? __longlong_as_double((long long)sh.bmax[h]) : -INFINITY;
      // group-of-8 reductions by DPP: quad_perm [1,0,3,2], [2,3,0,1], then
      // row_half_mirror (lane i of the eight with lane 7 - i)
      double mg = bmh;
      mg = fmax(mg, dpp_f64<0xB1, 0xf>(mg));
      mg = fmax(mg, dpp_f64<0x4E, 0xf>(mg));
      mg = fmax(mg, dpp_f64<0x141, 0xf>(mg));
      fpair = bmh == -INFINITY ? 0.0 : (bmh == mg ? 1.0 : exp(bmh - mg));
      double t = on ? (((sh.ps[0][h] + sh.ps[1][h]) + sh.ps[2][h]) + sh.ps[3][h]) * fpair : 0.0;
      int c = on ? sh.bcnt[h] : 0;
      t += dpp_f64<0xB1, 0xf>(t); c += dpp_i32<0xB1, 0xf>(0, c);
      t += dpp_f64<0x4E, 0xf>(t); c += dpp_i32<0x4E, 0xf>(0, c);
      t += dpp_f64<0x141, 0xf>(t); c += dpp_i32<0x141, 0xf>(0, c);
      const int src = 8 * min(lane, 7);
      m = __shfl(mg, src, 64);
      cs = __shfl(t, src, 64);
      cc = __shfl(c, src, 64);
    } else {
      // Hillis-Steele prefix: each step rescales the side with the smaller
      // maximum; an empty side (m = -inf) contributes nothing
      m = bm;
      cs = b < p.nrad ? ((sh.ps[0][b] + sh.ps[1][b]) + sh.ps[2][b]) + sh.ps[3][b] : 0.0;
      cc = b < p.nrad ? sh.bcnt[b] : 0;
      for (int o = 1; o < p.nrad; o <<= 1) {
        const double m2 = __shfl_up(m, o, 64), s2 = __shfl_up(cs, o, 64);
        const int c2 = __shfl_up(cc, o, 64);
        if (lane >= o) {
          const double mx = fmax(m, m2), mn = fmin(m, m2);
          const double f = mn == mx ? 1.0 : (mn == -INFINITY ? 0.0 : exp(mn - mx));
          cs = m >= m2 ? cs + s2 * f : cs * f + s2;
          m = mx;
          cc += c2;
        }
      }
    }
    const double lnu = (b < p.nrad && cc > 0) ? m + log(cs) : -INFINITY;
    const bool acc_ok = b < p.nrad && cc > 0 && lnu >= p.log_tnu;
    const uint64_t accm = __ballot(acc_ok);
    const int ncand = sh.red_i[0][0] + sh.red_i[1][0] + sh.red_i[2][0] + sh.red_i[3][0];
    const int ncom = sh.red_i[0][1] + sh.red_i[1][1] + sh.red_i[2][1] + sh.red_i[3][1];
    int layer = SKM_LAYER_IDL, ridx = p.nrad - 1, flags = relaxed_flag;
    bool want_hql = false;
    if (ncand == 0) {
      layer = SKM_LAYER_BRL;
      flags |= SKM_FLAG_NO_CAND;
    } else if (p.mode == SKM_MODE_FULL || gsel == SKM_LAYER_HQL) {
      want_hql = true;
    } else if (p.mode != SKM_MODE_PLAIN) {  // PROFILE, IDL, CNN (IDL choice or no network)
      if (accm) ridx = __ffsll((unsigned long long)accm) - 1;
      else want_hql = p.mode == SKM_MODE_PROFILE || (p.mode == SKM_MODE_CNN && !cnn);
    }
    if (want_hql) {
      // HQL's candidates: the complete ones, or every admissible one
      if ((p.hql_partial ? ncand : ncom) >= max(2, p.min_hql)) layer = SKM_LAYER_HQL;
      else flags |= SKM_FLAG_NO_HQL;
    }
    const double lnu_r = readlane_f64(lnu, ridx);      // ridx is uniform in the wave
    const double cs_r = readlane_f64(cs, ridx);
    const double m_r = readlane_f64(m, ridx);
    // weight of a candidate of bucket b <= ridx: term * exp(bm[b] - max over
    // buckets <= ridx); sums (cs_r) are relative to the same maximum
    if (r8) {
      if ((lane >> 3) == ridx && (lane & 7) < p.nrad) sh.fsc[lane & 7] = fpair;   // 0 past ridx
    } else if (lane < p.nrad) {
      sh.fsc[lane] = (lane <= ridx && bm != -INFINITY) ? (bm == m_r ? 1.0 : exp(bm - m_r)) : 0.0;
    }
    if (lane == 0) {
      sh.layer = layer; sh.radius_idx = ridx; sh.flags = flags;
      sh.n_cand = ncand; sh.n_complete = ncom;
      sh.lnu = ncand > 0 ? lnu_r : NAN;
      sh.den = cs_r;
      sh.xs = 16777216.0 / cs_r;
    }
  }
  __syncthreads();
  const int layer = sh.layer;
  if (layer == SKM_LAYER_HQL) {
    // HQL runs in the dense-algebra kernel after this one
    if (tid == 0) {
      write_info(a, i, bx, by, SKM_LAYER_HQL, round, sh.n_cand, sh.n_complete, W, sh.flags,
                 phi, n0, sh.lnu);
      a.bstate[i] = kNeedHql + round;
      if (pend) atomicAdd(pend, 1);                    // until the HQL kernel takes it
      a.hql_list[atomicAdd(&st->n_hql, 1)] = i;
    }
    return;
  }
  if (layer == SKM_LAYER_BRL) {
    write_const_block(a, p, i, x0, y0, mean, partial);
    if (tid == 0) {
      write_info(a, i, bx, by, SKM_LAYER_BRL, round, sh.n_cand, sh.n_complete, 0, sh.flags,
                 phi, n0, sh.lnu);
      a.bstate[i] = round;
    }
    return;
  }

  // 6. IDL weights (eq. slpe): term * fsc[b] = exp(ell - ell_max) in FP64,
  //    ell_max over the buckets <= ridx, rounded to FP32, for the candidates inside the
  //    accepted radius, compacted in raster order into (cand, dist) =
  //    (window offset, weight bits) after the scan's barriers.
  const int ridx = sh.radius_idx;
  {
    uint32_t o_r[KP], w_r[KP];
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      o_r[k] = 0u; w_r[k] = 0u;
      const int bj = cand_bucket(c_r[k]);
      if (t_r[k] >= 0.0 && bj <= ridx) {
        // a weight that underflows FP32 adds nothing and is left out
        const float w = (float)(t_r[k] * sh.fsc[bj]);
        o_r[k] = (uint32_t)cand_off(c_r[k]);
        w_r[k] = __float_as_uint(w);
        cnt += w_r[k] != 0u;
      }
    }
    int tot = 0;
    int pos = block_excl_scan(cnt, sh.scan, &tot);     // barriers inside
    uint32_t last_o = 0u;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (w_r[k] != 0u) { E.sel[pos] = make_uint2(o_r[k], w_r[k]); ++pos; last_o = o_r[k]; }
    }
    // padding to a multiple of 8, by the lane that wrote the last entry:
    // weight 0 at that entry's offset, whose prototype pixels are all known
    // (an unknown pixel read as binary16 is a NaN, and 0 * NaN is NaN)
    if (cnt > 0 && pos == tot)
      for (int e = tot; e < ((tot + 7) & ~7); ++e) E.sel[e] = make_uint2(last_o, 0u);
    if (tid == 0) sh.n_sel = tot;
  }
  __syncthreads();

  // 7. weighted average of the prototypes.  A lane owns two horizontally
  //    adjacent pixels, one window pair per candidate.  A pixel value 0..255
  //    in the low or high half of a pair, taken as the bits of a binary16
  //    number, is the subnormal value * 2^-24 (exact), so the mixed-precision
  //    FMA uses it without a conversion and the sums are scaled back by 2^24
  //    (exact) at the end.  Candidate groups of B*B/2 lanes split the
  //    selected candidates in blocks of 8; each lane of a group reads the
  //    same (offset, weight), an LDS broadcast.  Within a block FP32 FMA;
  //    blocks enter a Kahan-compensated sum; the groups' sums are added in
  //    FP64.
  {
    const int nsel = sh.n_sel;
    const int NP = B2 / 2;                  // pixel pairs per block (B is 4, 8 or 16)
    const int GG = kThreads / NP;           // candidate groups, at least 2
    const int h = tid / NP, q = tid - h * NP;
    const int py = (2 * q) / B, px = 2 * q - py * B;
    const uint32_t* wq = E.winp + (r + py) * Wp + (r + px);
    float acc0 = 0.f, acc1 = 0.f, comp0 = 0.f, comp1 = 0.f;
    for (int j0 = 8 * h; j0 < nsel; j0 += 8 * GG) {
      uint2 sv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) sv[t] = E.sel[j0 + t];
      uint32_t pv[8];
      float wv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        pv[t] = wq[(int)sv[t].x];
        wv[t] = __uint_as_float(sv[t].y);
      }
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        s0 = fmaf(wv[t], half_lo(pv[t]), s0);
        s1 = fmaf(wv[t], half_hi(pv[t]), s1);
      }
      float y = s0 - comp0, tt = acc0 + y;
      comp0 = (tt - acc0) - y; acc0 = tt;
      y = s1 - comp1; tt = acc1 + y;
      comp1 = (tt - acc1) - y; acc1 = tt;
    }
    *reinterpret_cast<float2*>(E.part + 2 * tid) = make_float2(acc0 - comp0, acc1 - comp1);
    __syncthreads();
    if (h == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int hh = 0; hh < GG; ++hh) {
        const float2 v = *reinterpret_cast<const float2*>(E.part + 2 * (hh * NP + q));
        t0 += (double)v.x;
        t1 += (double)v.y;
      }
      const double x0h = t0 * sh.xs, x1h = t1 * sh.xs;
      uint8_t* o = a.work + (size_t)(y0 + py) * p.stride + x0 + px;
      // the block's own pair in the window: received pixels are kept
      const uint32_t own = partial ? wq[W * Wp + W] : 0xffffffffu;
      if ((int16_t)(own & 0xffffu) < 0) o[0] = (uint8_t)fmin(fmax(floor(x0h + 0.5), 0.0), 255.0);
      if ((int16_t)(own >> 16) < 0) o[1] = (uint8_t)fmin(fmax(floor(x1h + 0.5), 0.0), 255.0);
      if (a.xhat && i < a.cap) {
        a.xhat[(size_t)i * B2 + 2 * q] = (float)x0h;
        a.xhat[(size_t)i * B2 + 2 * q + 1] = (float)x1h;
      }
    }
  }
  if (tid == 0)
    write_info(a, i, bx, by, SKM_LAYER_IDL, round, sh.n_cand, sh.n_complete, p.radii[ridx],
               sh.flags, phi, n0, sh.lnu);
  if (tid == 0) a.bstate[i] = round;
}

// one workgroup per lost block; the grid covers every cell.  Workgroups go
// round-robin to the 8 XCDs, so XCD x takes the x-th contiguous eighth of
// the (raster ordered) lost blocks: neighbouring windows share its L2.
template <int KP, int KR, bool FG>
__global__ __launch_bounds__(kThreads) void k_round_main(FrameArgs a, DevParams p, int dist_only) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BlockShared sh;
  const RoundState* st = a.st;
  if (st->remaining == 0) return;
  const int i = xcd_block(blockIdx.x, st->n_lost);
  if (i < 0) return;
  est_block<KP, KR, FG>(a, p, i, st->round, dist_only, lds_raw, sh, nullptr);
}

// -------------------------------------------------------------- finalize
// Blocks concealed in this round become known: their output pixels enter
// the value plane.  A workgroup takes kFinPer consecutive lost blocks at a
// time (their states read together, then one pixel per thread of each) and
// counts the blocks still pending and those left waiting for HQL; the
// workgroup that finishes last sets the next round's state.
constexpr int kFinPer = 16;

__global__ __launch_bounds__(kThreads) void k_round_finalize(FrameArgs a, DevParams p) {
  __shared__ int s_bs[kFinPer];
  __shared__ int s_vo[kFinPer], s_wo[kFinPer];
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  const int n_lost = st->n_lost, round = st->round;
  const int B = p.B, B2 = B * B, tid = threadIdx.x;
  const int lb = __ffs(B) - 1;                     // B is a power of two
  const int py = tid >> lb, px = tid & (B - 1);
  int pend = 0, hql = 0;
  for (int i0 = blockIdx.x * kFinPer; i0 < n_lost; i0 += gridDim.x * kFinPer) {
    if (tid < kFinPer) {
      const int i = i0 + tid;
      const int bs = i < n_lost ? a.bstate[i] : -1;
      const int cell = i < n_lost ? a.blk[i] : 0;
      const int by = cell / p.gw, bx = cell - by * p.gw;
      s_bs[tid] = bs;
      s_vo[tid] = by * B * p.width + bx * B;
      s_wo[tid] = by * B * p.stride + bx * B;
      pend += bs == 0;
      hql += bs >= kNeedHql;
    }
    __syncthreads();
    uint8_t v[kFinPer];
#pragma unroll
    for (int k = 0; k < kFinPer; ++k)
      v[k] = (tid < B2 && s_bs[k] == round) ? a.work[(size_t)s_wo[k] + (size_t)py * p.stride + px]
                                            : (uint8_t)0;
#pragma unroll
    for (int k = 0; k < kFinPer; ++k)
      if (tid < B2 && s_bs[k] == round)
        a.val[(size_t)s_vo[k] + (size_t)py * p.width + px] = (int16_t)v[k];
    __syncthreads();
  }
  // one 64-bit atomic per workgroup: pending count (bits 0-23), blocks
  // waiting for HQL (24-47) and a ticket (48-63); the workgroup that takes
  // the last ticket has every count in the value it gets back
  if (tid < 64) {
    pend = wave_sum(pend);
    hql = wave_sum(hql);
    if (tid == 0) {
      const unsigned long long mine =
          (unsigned long long)pend | ((unsigned long long)hql << 24) | (1ull << 48);
      const unsigned long long prev = atomicAdd(&st->round_acc, mine);
      if ((prev >> 48) + 1 == gridDim.x) {
        const unsigned long long tot = prev + mine;
        st->round_acc = 0ull;
        st->remaining = (int)(tot & 0xffffffull);
        st->round = round + 1;
        st->ctx_nq = 0; st->ctx_max = 0;
        if ((tot >> 24) & 0xffffffull) st->err |= kErrHqlPending;
        publish_state(a);
      }
    }
  }
}

// ------------------------------------------------------------------- fill
// After the round limit: context mean (or frame mean) for pending blocks.

__global__ void k_zero_fill(RoundState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { st->n_avail = 0; st->sum_avail = 0; }
}

__global__ __launch_bounds__(kThreads) void k_fill_stats(FrameArgs a, DevParams p) {
  __shared__ unsigned long long s_c[kThreads / 64], s_s[kThreads / 64];
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  unsigned long long cnt = 0, sum = 0;
  for (int y = blockIdx.x; y < p.height; y += gridDim.x) {
    for (int x = threadIdx.x; x < p.width; x += kThreads) {
      const int v = a.val[(size_t)y * p.width + x];
      if (v >= 0) { ++cnt; sum += (unsigned)v; }
    }
  }
  cnt = wave_sum(cnt);
  sum = wave_sum(sum);
  if (lane_id() == 0) { s_c[wave_id()] = cnt; s_s[wave_id()] = sum; }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long c = 0, s = 0;
    for (int w = 0; w < kThreads / 64; ++w) { c += s_c[w]; s += s_s[w]; }
    if (c) { atomicAdd(&st->n_avail, c); atomicAdd(&st->sum_avail, s); }
  }
}

__device__ __forceinline__ int block_sum_int(int v, int* s_red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) s_red[wave_id()] = v;
  __syncthreads();
  int t = 0;
  for (int w = 0; w < kThreads / 64; ++w) t += s_red[w];
  return t;
}

__global__ __launch_bounds__(kThreads) void k_fill(FrameArgs a, DevParams p) {
  __shared__ int s_red[kThreads / 64];
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  const int n_lost = st->n_lost, round = st->round;
  const int B = p.B, F = p.F, r = p.r;
  const double fmean = st->n_avail ? (double)st->sum_avail / (double)st->n_avail : 0.0;
  for (int i = blockIdx.x; i < n_lost; i += gridDim.x) {
    if (a.bstate[i] != 0) continue;
    const int cell = a.blk[i];
    const int by = cell / p.gw, bx = cell - by * p.gw;
    const int xr = bx * B - r, yr = by * B - r;
    // context: the footprint, with the block's own received pixels (counted
    // again in bits 16.. to flag a partly received block)
    int c = 0, s = 0;
    for (int pos = threadIdx.x; pos < F * F; pos += blockDim.x) {
      const int fy = pos / F, fx = pos - fy * F;
      const bool own = fy >= r && fy < r + B && fx >= r && fx < r + B;
      const int gy = yr + fy, gx = xr + fx;
      if (gy >= 0 && gy < p.height && gx >= 0 && gx < p.width) {
        const int v = a.val[(size_t)gy * p.width + gx];
        if (v >= 0) { c += own ? 1 + (1 << 16) : 1; s += v; }
      }
    }
    c = block_sum_int(c, s_red);
    s = block_sum_int(s, s_red);
    const bool partial = (c >> 16) > 0;
    c &= 0xffff;
    const double v = c > 0 ? (double)s / (double)c : fmean;
    write_const_block(a, p, i, bx * B, by * B, v, partial);
    if (threadIdx.x == 0) {
      write_info(a, i, bx, by, SKM_LAYER_FILL, round, -1, -1, 0,
                 c > 0 ? 0 : SKM_FLAG_EMPTY_CTX, 0, c, NAN);
      a.bstate[i] = round;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ batched
// Batched pipeline over the nf frames of a BatchArgs (equal size and
// parameters p).  Items are the (frame, lost block) pairs in frame order;
// cum[f] is the index of frame f's first item.  Persistent kernels give XCD x
// the x-th contiguous eighth of the items, as the single-frame kernels do
// per frame.

// items of this workgroup's XCD eighth: first, end, stride (grid a multiple
// of 8); `sub` of `lanes_per_wg` sub-units (waves) of the workgroup
struct XcdRange { int first, end, step; };
static __device__ __forceinline__ XcdRange xcd_items(int total, int lanes_per_wg, int sub) {
  const int per8 = (total + 7) >> 3, xcd = blockIdx.x & 7;
  const int g0 = min(total, xcd * per8);
  XcdRange r;
  r.first = g0 + (int)(blockIdx.x >> 3) * lanes_per_wg + sub;
  r.end = min(total, g0 + per8);
  r.step = (int)(gridDim.x >> 3) * lanes_per_wg;
  return r;
}

static __device__ __forceinline__ void publish_batch(const BatchArgs& b) {
  if (!b.hbs) return;
  b.hbs->total = b.bs->total;
  b.hbs->remaining = b.bs->remaining;
  b.hbs->err = b.bs->err;
}

// Loss geometry of every frame: init_wgs(p) workgroups per frame.  The
// workgroup that lists the last frame's cells writes the item offsets cum[]
// and the batch totals.
__global__ __launch_bounds__(kThreads) void k_init_b(BatchArgs b, DevParams p) {
  __shared__ int s_lastf;
  const int wpf = init_wgs(p), gx = init_wg_x(p);
  const int f = (int)blockIdx.x / wpf, local = (int)blockIdx.x - f * wpf;
  const FrameArgs a = batch_frame(b, f);
  if (!init_body(a, p, local % gx, local / gx, (unsigned)wpf)) return;
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned t = atomicAdd(&b.bs->frames_done, 1u);
    s_lastf = t + 1 == (unsigned)b.nf;
    if (s_lastf) atomicExch(&b.bs->frames_done, 0u);
  }
  __syncthreads();
  if (!s_lastf || threadIdx.x != 0) return;
  __threadfence();
  int acc = 0, rem = 0, err = 0;
  for (int k = 0; k < b.nf; ++k) {
    RoundState* sk = b.a0.st + k;
    b.cum[k] = acc;
    acc += __hip_atomic_load(&sk->n_lost, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int ek = __hip_atomic_load(&sk->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ek) {
      // a frame with a geometry error runs no round (its status reports it)
      sk->remaining = 0;
      publish_state_to(sk, b.a0.hstate ? b.a0.hstate + k : nullptr);
    }
    rem += __hip_atomic_load(&sk->remaining, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    err |= ek;
  }
  b.cum[b.nf] = acc;
  b.bs->total = acc;
  b.bs->remaining = rem;
  b.bs->err = err;
  publish_batch(b);
}

// Round preparation of every frame: one wave per item; each wave adds its
// (nq, mx) to a frame's context rule when it moves to another frame.
__global__ __launch_bounds__(kThreads) void k_round_prep_b(BatchArgs b, DevParams p) {
  if (b.bs->remaining == 0) return;
  if (blockIdx.x == 0)
    for (int f = threadIdx.x; f < b.nf; f += kThreads) b.a0.st[f].n_hql = 0;
  const int lane = lane_id(), wave = wave_id();
  const XcdRange R = xcd_items(b.bs->total, kThreads / 64, wave);
  if (R.first >= R.end) return;
  int f = frame_of(b.cum, b.nf, R.first);
  FrameArgs a = batch_frame(b, f);
  int nq = 0, mx = 0;
  for (int g = R.first; g < R.end; g += R.step) {
    if (g >= b.cum[f + 1]) {
      if (lane == 0) note_context_rule(a.st, nq, mx);
      nq = 0; mx = 0;
      while (g >= b.cum[f + 1]) ++f;
      a = batch_frame(b, f);
    }
    const int i = g - b.cum[f];
    if (a.st->remaining == 0 || a.bstate[i] != 0) continue;
    prep_one(a, p, i, lane, nq, mx);
  }
  if (lane == 0) note_context_rule(a.st, nq, mx);
}

// Estimation over every frame's items: frame f owns workgroups
// [f cpad, (f + 1) cpad), cpad = the cell count rounded up to a multiple of
// 8, and maps them to its lost blocks as the single-frame kernel does (XCD x
// takes the x-th contiguous eighth).  A persistent loop over the items was
// measured first: carrying the frame's buffers and parameters across
// iterations spilled the scalar registers into 250 VGPRs (one wave per SIMD).
template <int KP, int KR, bool FG>
__global__ __launch_bounds__(kThreads) void k_round_main_b(BatchArgs b, DevParams p) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BlockShared sh;
  const int cpad = (p.gh * p.gw + 7) & ~7;
  const int f = (int)blockIdx.x / cpad;
  const FrameArgs a = batch_frame(b, f);
  const RoundState* st = a.st;
  if (st->remaining == 0) return;
  const int i = xcd_block((int)blockIdx.x - f * cpad, st->n_lost);
  if (i < 0) return;
  est_block<KP, KR, FG>(a, p, i, st->round, 0, lds_raw, sh, &b.bs->pending);
}

// Finalize of every frame: the concealed blocks of the round enter the value
// planes; pending and HQL-waiting blocks are counted per frame (one atomic
// per run of a frame in a step); the workgroup that finishes last closes the
// round of every frame that had one and publishes the states.
__global__ __launch_bounds__(kThreads) void k_round_finalize_b(BatchArgs b, DevParams p) {
  __shared__ int s_bs[kFinPer], s_round[kFinPer], s_f[kFinPer], s_cnt[kFinPer];
  __shared__ int s_vo[kFinPer], s_wo[kFinPer];
  __shared__ int s_last, s_red[2][kThreads / 64];
  if (b.bs->remaining == 0) return;
  const int tid = threadIdx.x;
  if (__hip_atomic_load(&b.bs->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    // no block of any frame is left pending: every frame that had a round
    // is complete, and no later round reads the value planes
    if (blockIdx.x != 0) return;
    int err = 0;
    for (int f = tid; f < b.nf; f += kThreads) {
      const FrameArgs a = batch_frame(b, f);
      RoundState* st = a.st;
      if (st->remaining != 0) {
        st->remaining = 0;
        st->round = st->round + 1;
        st->ctx_nq = 0; st->ctx_max = 0;
        publish_state(a);
      }
      err |= st->err;
    }
    for (int o = 32; o > 0; o >>= 1) err |= __shfl_xor(err, o, 64);
    if (lane_id() == 0) s_red[1][wave_id()] = err;
    __syncthreads();
    if (tid == 0) {
      int ee = 0;
      for (int w = 0; w < kThreads / 64; ++w) ee |= s_red[1][w];
      b.bs->remaining = 0;
      b.bs->err = ee;
      publish_batch(b);
    }
    return;
  }
  const int total = b.bs->total;
  const int B = p.B, B2 = B * B;
  const int lb = __ffs(B) - 1;
  const int py = tid >> lb, px = tid & (B - 1);
  for (int g0 = blockIdx.x * kFinPer; g0 < total; g0 += gridDim.x * kFinPer) {
    if (tid < kFinPer) {
      const int g = g0 + tid;
      int bs = -1, f = -1, rnd = 0, cnt = 0;
      if (g < total) {
        f = frame_of(b.cum, b.nf, g);
        const FrameArgs a = batch_frame(b, f);
        if (a.st->remaining != 0) {
          const int i = g - b.cum[f];
          bs = a.bstate[i];
          rnd = a.st->round;
          const int cell = a.blk[i];
          const int by = cell / p.gw, bx = cell - by * p.gw;
          s_vo[tid] = by * B * p.width + bx * B;
          s_wo[tid] = by * B * p.stride + bx * B;
          cnt = (bs == 0 ? 1 : 0) | (bs >= kNeedHql ? 1 << 24 : 0);
        } else {
          f = -1;
        }
      }
      s_bs[tid] = bs; s_round[tid] = rnd; s_f[tid] = f; s_cnt[tid] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
      // one atomic per run of equal frames in this step
      int k = 0;
      while (k < kFinPer) {
        const int f = s_f[k];
        unsigned long long c = 0;
        int e = k;
        while (e < kFinPer && s_f[e] == f) c += (unsigned long long)s_cnt[e++];
        if (f >= 0 && c) atomicAdd(&b.a0.st[f].round_acc, c);
        k = e;
      }
    }
    uint8_t v[kFinPer];
#pragma unroll
    for (int k = 0; k < kFinPer; ++k) {
      const bool cpy = tid < B2 && s_bs[k] > 0 && s_bs[k] == s_round[k];
      v[k] = cpy ? b.io[s_f[k]].out[(size_t)s_wo[k] + (size_t)py * p.stride + px] : (uint8_t)0;
    }
#pragma unroll
    for (int k = 0; k < kFinPer; ++k) {
      const bool cpy = tid < B2 && s_bs[k] > 0 && s_bs[k] == s_round[k];
      if (cpy)
        b.a0.val[(size_t)s_f[k] * b.val_stride + (size_t)s_vo[k] + (size_t)py * p.width + px] =
            (int16_t)v[k];
    }
    __syncthreads();
  }
  if (tid == 0) {
    __threadfence();
    const unsigned t = atomicAdd(&b.bs->fin_ticket, 1u);
    s_last = t + 1 == gridDim.x;
    if (s_last) atomicExch(&b.bs->fin_ticket, 0u);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  int rem = 0, err = 0;
  for (int f = tid; f < b.nf; f += kThreads) {
    const FrameArgs a = batch_frame(b, f);
    RoundState* st = a.st;
    if (st->remaining == 0) { err |= st->err; continue; }
    const unsigned long long tot =
        __hip_atomic_load(&st->round_acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st->round_acc = 0ull;
    st->remaining = (int)(tot & 0xffffffull);
    st->round = st->round + 1;
    st->ctx_nq = 0; st->ctx_max = 0;
    if ((tot >> 24) & 0xffffffull) st->err |= kErrHqlPending;
    // a frame with an error stops here (its status reports it; the
    // single-frame pipeline stops at the same point)
    if (st->err) st->remaining = 0;
    publish_state(a);
    rem += st->remaining;
    err |= st->err;
  }
  rem = wave_sum(rem);
  int e = err;
  for (int o = 32; o > 0; o >>= 1) e |= __shfl_xor(e, o, 64);
  if (lane_id() == 0) { s_red[0][wave_id()] = rem; s_red[1][wave_id()] = e; }
  __syncthreads();
  if (tid == 0) {
    int r = 0, ee = 0;
    for (int w = 0; w < kThreads / 64; ++w) { r += s_red[0][w]; ee |= s_red[1][w]; }
    b.bs->remaining = r;
    b.bs->err = ee;
    b.bs->pending = 0;                     // counted afresh by the next round
    publish_batch(b);
  }
}

// -------------------------------------------------------------- launchers

static int clamp_grid(long long g, int hi) {
  return (int)(g < 1 ? 1 : (g > hi ? hi : g));
}

hipError_t launch_init(const FrameArgs& a, const DevParams& p, hipStream_t s) {
  dim3 g((p.width + 4 * kThreads - 1) / (4 * kThreads), (p.height + p.B - 1) / p.B);
  hipLaunchKernelGGL(k_init, g, dim3(kThreads), 0, s, a, p);
  return hipGetLastError();
}

static hipError_t launch_main(const FrameArgs& a, const DevParams& p, int max_blocks,
                              int dist_only, hipStream_t s) {
  const size_t lds = main_lds_bytes(p);
  const int grid = ((max_blocks < 1 ? 1 : max_blocks) + 7) / 8 * 8;   // xcd_block cover
  const int per = (p.MC + kThreads - 1) / kThreads;
  const bool fg = p.B == Geom16::kB && p.r == Geom16::kR && p.W == Geom16::kW;
  if (fg && per <= 6 && p.nrad <= 8)
    hipLaunchKernelGGL((k_round_main<6, 8, true>), dim3(grid), dim3(kThreads), lds, s, a, p,
                       dist_only);
  else if (per <= 6 && p.nrad <= 8)
    hipLaunchKernelGGL((k_round_main<6, 8, false>), dim3(grid), dim3(kThreads), lds, s, a, p,
                       dist_only);
  else if (per <= 9 && p.nrad <= 8)
    hipLaunchKernelGGL((k_round_main<9, 8, false>), dim3(grid), dim3(kThreads), lds, s, a, p,
                       dist_only);
  else
    hipLaunchKernelGGL((k_round_main<kMaxPer, kMaxRadii, false>), dim3(grid), dim3(kThreads), lds,
                       s, a, p, dist_only);
  return hipGetLastError();
}

int prep_grid_for(int max_blocks) {
  const int g = clamp_grid((max_blocks + 3) / 4, kPrepGridMax);
  return g >= 8 ? (g + 7) / 8 * 8 : g;       // whole XCD groups (kPrepGridMax is one)
}

hipError_t launch_prep(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_round_prep, dim3(p.prep_grid), dim3(kThreads), 0, s, a, p);
  return hipGetLastError();
}

hipError_t launch_est(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s) {
  return launch_main(a, p, max_blocks, 0, s);
}

hipError_t launch_finalize(const FrameArgs& a, const DevParams& p, int max_blocks,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_round_finalize, dim3(clamp_grid((max_blocks + kFinPer - 1) / kFinPer, 256)),
                     dim3(kThreads), 0, s, a, p);
  return hipGetLastError();
}

hipError_t launch_dist(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s) {
  return launch_main(a, p, max_blocks, 1, s);
}

hipError_t launch_fill(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_fill, dim3(1), dim3(64), 0, s, a.st);
  hipLaunchKernelGGL(k_fill_stats, dim3(clamp_grid(p.height, 1024)), dim3(kThreads), 0, s, a, p);
  hipLaunchKernelGGL(k_fill, dim3(clamp_grid(max_blocks, 2048)), dim3(kThreads), 0, s, a, p);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_zero_words(unsigned int* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    p[i] = 0u;
}

hipError_t launch_zero_words(unsigned int* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3(clamp_grid((long long)((n + kThreads - 1) / kThreads), 256)),
                     dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

// Estimation kernel variants: 0 = <6, 8> with the compile-time unit offsets
// of the 16 x 16 / ring 4 / window 24 geometry, 1 = <6, 8>, 2 = <9, 8>,
// 3 = <17, 16> (candidate slices per thread, expansion radii).  The first
// variant written is the one launch_main uses.
int est_variants(const DevParams& p, int* out) {
  const int per = (p.MC + kThreads - 1) / kThreads;
  const bool fg = p.B == Geom16::kB && p.r == Geom16::kR && p.W == Geom16::kW;
  int n = 0;
  if (fg && per <= 6 && p.nrad <= 8) out[n++] = 0;
  if (per <= 6 && p.nrad <= 8) out[n++] = 1;
  if (per <= 9 && p.nrad <= 8) out[n++] = 2;
  out[n++] = 3;
  return n;
}

hipError_t launch_init_b(const BatchArgs& b, const DevParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_init_b, dim3(b.nf * init_wgs(p)), dim3(kThreads), 0, s, b, p);
  return hipGetLastError();
}

hipError_t launch_prep_b(const BatchArgs& b, const DevParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_round_prep_b, dim3((grid + 7) / 8 * 8), dim3(kThreads), 0, s, b, p);
  return hipGetLastError();
}

hipError_t launch_est_b(const BatchArgs& b, const DevParams& p, int variant, hipStream_t s) {
  const size_t lds = main_lds_bytes(p);
  const dim3 g(b.nf * ((p.gh * p.gw + 7) & ~7));
  switch (variant) {
    case 0: hipLaunchKernelGGL((k_round_main_b<6, 8, true>), g, dim3(kThreads), lds, s, b, p); break;
    case 1: hipLaunchKernelGGL((k_round_main_b<6, 8, false>), g, dim3(kThreads), lds, s, b, p); break;
    case 2: hipLaunchKernelGGL((k_round_main_b<9, 8, false>), g, dim3(kThreads), lds, s, b, p); break;
    default:
      hipLaunchKernelGGL((k_round_main_b<kMaxPer, kMaxRadii, false>), g, dim3(kThreads), lds, s, b,
                         p);
  }
  return hipGetLastError();
}

hipError_t launch_finalize_b(const BatchArgs& b, const DevParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_round_finalize_b, dim3(grid < 1 ? 1 : grid), dim3(kThreads), 0, s, b, p);
  return hipGetLastError();
}

hipError_t set_main_lds_limit(size_t bytes) {
  const void* fns[8] = {(const void*)k_round_main<6, 8, true>, (const void*)k_round_main<6, 8, false>,
                        (const void*)k_round_main<9, 8, false>,
                        (const void*)k_round_main<kMaxPer, kMaxRadii, false>,
                        (const void*)k_round_main_b<6, 8, true>,
                        (const void*)k_round_main_b<6, 8, false>,
                        (const void*)k_round_main_b<9, 8, false>,
                        (const void*)k_round_main_b<kMaxPer, kMaxRadii, false>};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace skm
