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
#include <math.h>

#include "skm_internal.h"

namespace skm {

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// Merge two (max, sum of exp(x - max)) pairs.  Order-fixed callers make the
// result deterministic.
__device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2) {
  if (m2 == -INFINITY) return;
  if (m == -INFINITY) { m = m2; s = s2; return; }
  if (m2 > m) { s = s * exp(m - m2) + s2; m = m2; }
  else        { s = s + s2 * exp(m2 - m); }
}

__device__ __forceinline__ void wave_lse(double& m, double& s) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double m2 = __shfl_xor(m, o, 64);
    double s2 = __shfl_xor(s, o, 64);
    // both partners must compute the same merge irrespective of role:
    // merge in lane order (lower lane first) so that the result is symmetric.
    bool lower = (lane_id() & o) == 0;
    double ma = lower ? m : m2, sa = lower ? s : s2;
    double mb = lower ? m2 : m, sb = lower ? s2 : s;
    lse_merge(ma, sa, mb, sb);
    m = ma; s = sa;
  }
}

// ---------------------------------------------------------- state / setup

__global__ void k_zero_state(RoundState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->n_lost = 0; st->remaining = 0; st->remaining_acc = 0; st->nq = 0;
    st->maxm0 = 0; st->round = 1; st->err = 0; st->done_wgs = 0;
    st->n_avail = 0; st->sum_avail = 0;
  }
}

// avail = mask == 0; work = avail ? frame : 128.  Lost pixels outside the full
// cell grid are an error.  Counts the received pixels.
__global__ __launch_bounds__(kThreads) void k_init(FrameArgs a, DevParams p) {
  const long long npx = (long long)p.width * p.height;
  const int gxB = p.gw * p.B, gyB = p.gh * p.B;
  unsigned long long cnt = 0;
  int bad = 0;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < npx;
       idx += (long long)gridDim.x * blockDim.x) {
    int y = (int)(idx / p.width), x = (int)(idx - (long long)y * p.width);
    size_t off = (size_t)y * p.stride + x;
    bool lost = a.mask[off] != 0;
    uint8_t v = lost ? (uint8_t)128 : a.frame[off];
    a.work[off] = v;
    a.avail[idx] = lost ? 0 : 1;
    cnt += lost ? 0 : 1;
    if (lost && (x >= gxB || y >= gyB)) bad = 1;
  }
  cnt = wave_sum(cnt);
  bad = wave_max(bad);
  if (lane_id() == 0) {
    if (cnt) atomicAdd(&a.st->n_avail, cnt);
    if (bad) atomicOr(&a.st->err, kErrPartial);
  }
}

// one thread per full cell: lost iff every pixel is lost; partly lost = error
__global__ __launch_bounds__(kThreads) void k_cells(FrameArgs a, DevParams p) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p.gh * p.gw) return;
  int by = c / p.gw, bx = c - by * p.gw;
  int n = 0;
  for (int i = 0; i < p.B; ++i) {
    const uint8_t* row = a.mask + (size_t)(by * p.B + i) * p.stride + bx * p.B;
    for (int j = 0; j < p.B; ++j) n += row[j] != 0;
  }
  a.cell_lost[c] = n == p.B * p.B;
  if (n != 0 && n != p.B * p.B) atomicOr(&a.st->err, kErrPartial);
}

// single workgroup of 1024: ordered compaction of lost cells
__global__ __launch_bounds__(1024) void k_compact(FrameArgs a, DevParams p) {
  __shared__ int s_cnt[1024];
  const int ncell = p.gh * p.gw;
  const int tid = threadIdx.x;
  const int chunk = (ncell + 1023) / 1024;
  const int c0 = min(ncell, tid * chunk), c1 = min(ncell, c0 + chunk);
  int n = 0;
  for (int c = c0; c < c1; ++c) n += a.cell_lost[c];
  s_cnt[tid] = n;
  __syncthreads();
  // Hillis-Steele inclusive scan
  for (int o = 1; o < 1024; o <<= 1) {
    int v = tid >= o ? s_cnt[tid - o] : 0;
    __syncthreads();
    s_cnt[tid] += v;
    __syncthreads();
  }
  int pos = s_cnt[tid] - n;
  for (int c = c0; c < c1; ++c) {
    if (a.cell_lost[c]) {
      a.blk[pos] = c;
      a.bstate[pos] = 0;
      ++pos;
    }
  }
  if (tid == 1023) {
    a.st->n_lost = s_cnt[1023];
    a.st->remaining = s_cnt[1023];
    a.st->round = 1;
  }
}

// ------------------------------------------------------------- round prep
// one wave per pending block: |m0| = known in-frame ring pixels
__global__ __launch_bounds__(kThreads) void k_round_prep(FrameArgs a, DevParams p) {
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) { st->remaining_acc = 0; st->done_wgs = 0; }
  const int n_lost = st->n_lost;
  const int nwaves = gridDim.x * (blockDim.x / 64);
  const int F = p.F;
  for (int i = blockIdx.x * (blockDim.x / 64) + wave_id(); i < n_lost; i += nwaves) {
    if (a.bstate[i] != 0) continue;
    int cell = a.blk[i];
    int by = cell / p.gw, bx = cell - by * p.gw;
    int x0 = bx * p.B - p.r, y0 = by * p.B - p.r;
    int c = 0;
    for (int pos = lane_id(); pos < F * F; pos += 64) {
      int fy = pos / F, fx = pos - fy * F;
      bool ring = fy < p.r || fy >= p.r + p.B || fx < p.r || fx >= p.r + p.B;
      int gy = y0 + fy, gx = x0 + fx;
      if (ring && gy >= 0 && gy < p.height && gx >= 0 && gx < p.width)
        c += a.avail[(size_t)gy * p.width + gx];
    }
    c = wave_sum(c);
    if (lane_id() == 0) {
      a.m0cnt[i] = c;
      if (c >= p.r * p.B) atomicAdd(&st->nq, 1);
      atomicMax(&st->maxm0, c);
    }
  }
}

// ----------------------------------------------------------- main kernel

struct MainLds {
  double* ell;          // [ND] log raw weight, -inf if not admissible
  uint64_t* rowbits;    // [Wd*2] availability bits of each window row
  int* dval;            // [ND] distance (reused as float weights)
  uint32_t* q;          // [F*F] query ring: offset | value << 16
  uint16_t* list;       // [ND] admissible-prototype displacement indices
  uint16_t* nval;       // [ND] overlap counts
  int16_t* win;         // [Wd*Wd] window pixels, -1 = unknown
};

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

__host__ __device__ inline size_t main_lds_layout(const DevParams& p, size_t* offs) {
  size_t o = 0;
  offs[0] = o; o = align_up(o + sizeof(double) * p.ND, 16);
  offs[1] = o; o = align_up(o + sizeof(uint64_t) * p.Wd * 2, 16);
  offs[2] = o; o = align_up(o + sizeof(int) * p.ND, 16);
  offs[3] = o; o = align_up(o + sizeof(uint32_t) * p.F * p.F, 16);
  offs[4] = o; o = align_up(o + sizeof(uint16_t) * p.ND, 16);
  offs[5] = o; o = align_up(o + sizeof(uint16_t) * p.ND, 16);
  offs[6] = o; o = align_up(o + sizeof(int16_t) * p.Wd * p.Wd, 16);
  return o;
}

size_t main_lds_bytes(const DevParams& p) {
  size_t offs[8];
  return main_lds_layout(p, offs);
}

// B consecutive availability bits of window row `row` starting at column c
__device__ __forceinline__ bool row_run_ok(const uint64_t* rb, int row, int c, int B) {
  uint64_t lo = rb[2 * row], hi = rb[2 * row + 1];
  uint64_t v = c == 0 ? lo : (c < 64 ? (lo >> c) | (hi << (64 - c)) : hi >> (c - 64));
  uint64_t m = (B >= 64) ? ~0ull : ((1ull << B) - 1ull);
  return (v & m) == m;
}

__device__ __forceinline__ int block_sum_int(int v, int* s_red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) s_red[wave_id()] = v;
  __syncthreads();
  int t = s_red[0] + s_red[1] + s_red[2] + s_red[3];
  return t;
}

__device__ __forceinline__ double block_sum_double(double v, double* s_red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) s_red[wave_id()] = v;
  __syncthreads();
  return ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
}

__device__ __forceinline__ void block_lse(double& m, double& s, double* s_m, double* s_s) {
  wave_lse(m, s);
  __syncthreads();
  if (lane_id() == 0) { s_m[wave_id()] = m; s_s[wave_id()] = s; }
  __syncthreads();
  m = s_m[0]; s = s_s[0];
  for (int w = 1; w < kThreads / 64; ++w) lse_merge(m, s, s_m[w], s_s[w]);
}

// Per-block scratch shared by the whole workgroup.
struct BlockShared {
  int n0, phi, sum;
  int M;                      // admissible-prototype candidates
  int layer, radius_idx, flags, n_cand, n_complete;
  double lnu;
  int red_i[4];
  double red_d[4], red_m[4], red_s[4];
  double lse_m[kMaxRadii], lse_s[kMaxRadii];
  int lse_c[kMaxRadii];
  int scan[kThreads];
  double part[kThreads];
};

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

__global__ __launch_bounds__(kThreads) void k_round_main(FrameArgs a, DevParams p, int dist_only) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BlockShared sh;
  RoundState* st = a.st;
  const int remaining = st->remaining;
  if (remaining == 0) return;
  const int n_lost = st->n_lost, nq = st->nq, maxm0 = st->maxm0, round = st->round;
  if (!dist_only && nq == 0 && maxm0 == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&st->err, kErrNoContext);
    return;
  }
  size_t offs[8];
  main_lds_layout(p, offs);
  MainLds L;
  L.ell = (double*)(lds_raw + offs[0]);
  L.rowbits = (uint64_t*)(lds_raw + offs[1]);
  L.dval = (int*)(lds_raw + offs[2]);
  L.q = (uint32_t*)(lds_raw + offs[3]);
  L.list = (uint16_t*)(lds_raw + offs[4]);
  L.nval = (uint16_t*)(lds_raw + offs[5]);
  L.win = (int16_t*)(lds_raw + offs[6]);

  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int B = p.B, r = p.r, W = p.W, Wd = p.Wd, F = p.F, ND = p.ND, D2 = 2 * W + 1;
  const int B2 = B * B;

  for (int i = blockIdx.x; i < n_lost; i += gridDim.x) {
    if (a.bstate[i] != 0) continue;
    if (!dist_only) {
      int m0c = a.m0cnt[i];
      bool elig = nq > 0 ? (m0c >= r * B) : (m0c == maxm0);
      if (!elig) continue;
    }
    const int cell = a.blk[i];
    const int by = cell / p.gw, bx = cell - by * p.gw;
    const int x0 = bx * B, y0 = by * B;
    const int ox = x0 - r - W, oy = y0 - r - W;

    // 1. stage the search window (coalesced row reads)
    for (int idx = tid; idx < Wd * Wd; idx += kThreads) {
      int wy = idx / Wd, wx = idx - wy * Wd;
      int gy = oy + wy, gx = ox + wx;
      int v = -1;
      if (gx >= 0 && gx < p.width && gy >= 0 && gy < p.height) {
        if (a.avail[(size_t)gy * p.width + gx]) v = a.work[(size_t)gy * p.stride + gx];
      }
      L.win[idx] = (int16_t)v;
    }
    __syncthreads();

    // 2. availability bitmask per window row; 3. context list (wave 0)
    for (int row = wave; row < Wd; row += kThreads / 64) {
      bool b0 = lane < Wd && L.win[row * Wd + lane] >= 0;
      bool b1 = 64 + lane < Wd && L.win[row * Wd + 64 + lane] >= 0;
      uint64_t lo = __ballot(b0), hi = __ballot(b1);
      if (lane == 0) { L.rowbits[2 * row] = lo; L.rowbits[2 * row + 1] = hi; }
    }
    if (wave == 0) {
      int n = 0, vmin = 255, vmax = 0, vsum = 0;
      for (int base = 0; base < F * F; base += 64) {
        int pos = base + lane;
        int fy = pos / F, fx = pos - fy * F;
        bool ring = pos < F * F && (fy < r || fy >= r + B || fx < r || fx >= r + B);
        int v = ring ? L.win[(W + fy) * Wd + W + fx] : -1;
        bool ok = v >= 0;
        uint64_t m = __ballot(ok);
        int rank = __popcll(m & ((1ull << lane) - 1ull));
        if (ok) {
          L.q[n + rank] = (uint32_t)(fy * Wd + fx) | ((uint32_t)v << 16);
          vmin = min(vmin, v); vmax = max(vmax, v); vsum += v;
        }
        n += __popcll(m);
      }
      vmin = wave_min(vmin); vmax = wave_max(vmax); vsum = wave_sum(vsum);
      if (lane == 0) { sh.n0 = n; sh.phi = n > 0 ? vmax - vmin : 0; sh.sum = vsum; }
    }
    __syncthreads();
    const int n0 = sh.n0, phi = sh.phi;
    const double mean = n0 > 0 ? (double)sh.sum / (double)n0 : 0.0;
    const int relaxed_flag = (!dist_only && nq == 0) ? SKM_FLAG_CTX_RELAXED : 0;

    // BRL gate: context mean for every pixel of the block
    const bool profile_like = p.mode == SKM_MODE_PROFILE || p.mode == SKM_MODE_CNN;
    if (!dist_only && (p.mode == SKM_MODE_BRL || (profile_like && (double)phi <= p.t_phi))) {
      for (int pix = tid; pix < B2; pix += kThreads) {
        int py = pix / B, px = pix - py * B;
        double v = floor(mean + 0.5);
        v = fmin(fmax(v, 0.0), 255.0);
        a.work[(size_t)(y0 + py) * p.stride + x0 + px] = (uint8_t)v;
        if (a.xhat && i < a.cap) a.xhat[(size_t)i * B2 + pix] = (float)mean;
      }
      if (tid == 0) {
        write_info(a, i, bx, by, SKM_LAYER_BRL, round, -1, -1, 0, relaxed_flag, phi, n0, NAN);
        a.bstate[i] = round;
      }
      __syncthreads();
      continue;
    }

    // 4. admissible prototypes (in frame, fully received), raster order
    {
      const int center = ND / 2;
      const int chunk = (ND + kThreads - 1) / kThreads;
      const int t0 = min(ND, tid * chunk), t1 = min(ND, t0 + chunk);
      int cnt = 0;
      for (int t = t0; t < t1; ++t) {
        if (t == center) continue;
        int dy = t / D2 - W, dx = t - (t / D2) * D2 - W;
        int wy = W + r + dy, wx = W + r + dx;
        bool ok = true;
        for (int k = 0; k < B && ok; ++k) ok = row_run_ok(L.rowbits, wy + k, wx, B);
        cnt += ok;
      }
      sh.scan[tid] = cnt;
      __syncthreads();
      for (int o = 1; o < kThreads; o <<= 1) {
        int v = tid >= o ? sh.scan[tid - o] : 0;
        __syncthreads();
        sh.scan[tid] += v;
        __syncthreads();
      }
      int pos = sh.scan[tid] - cnt;
      for (int t = t0; t < t1; ++t) {
        if (t == center) continue;
        int dy = t / D2 - W, dx = t - (t / D2) * D2 - W;
        int wy = W + r + dy, wx = W + r + dx;
        bool ok = true;
        for (int k = 0; k < B && ok; ++k) ok = row_run_ok(L.rowbits, wy + k, wx, B);
        if (ok) L.list[pos++] = (uint16_t)t;
      }
      if (tid == kThreads - 1) sh.M = sh.scan[kThreads - 1];
      __syncthreads();
    }
    const int M = sh.M;

    // 5. exact integer distances over the ring pixels known in both rings
    const int nmin = max(1, (p.min_pct * n0 + 99) / 100);
    const double inv2s = 2.0 * p.sigma2;
    for (int j = tid; j < M; j += kThreads) {
      int t = L.list[j];
      int dy = t / D2 - W, dx = t - (t / D2) * D2 - W;
      int base = (W + dy) * Wd + (W + dx);
      int d = 0, n = 0;
      for (int k = 0; k < n0; ++k) {
        uint32_t qq = L.q[k];
        int pv = L.win[base + (int)(qq & 0xffffu)];
        if (pv >= 0) {
          int df = (int)(qq >> 16) - pv;
          d += df * df;
          ++n;
        }
      }
      bool ok = n >= nmin;
      L.dval[j] = ok ? d : -1;
      L.nval[j] = (uint16_t)n;
      L.ell[j] = ok ? -((double)d / (double)n) / inv2s : -INFINITY;
    }
    __syncthreads();

    if (dist_only) {
      int* drow = a.dist + (size_t)i * ND;
      int* crow = a.cnt + (size_t)i * ND;
      for (int t = tid; t < ND; t += kThreads) { drow[t] = -1; crow[t] = 0; }
      __syncthreads();
      for (int j = tid; j < M; j += kThreads) {
        if (L.dval[j] >= 0) { drow[L.list[j]] = L.dval[j]; crow[L.list[j]] = L.nval[j]; }
      }
      __syncthreads();
      continue;
    }

    // 6. candidate counts and log nu(rho) for every expansion radius
    {
      int nc = 0, ncomp = 0;
      for (int j = tid; j < M; j += kThreads) {
        if (L.dval[j] >= 0) { ++nc; ncomp += (L.nval[j] == n0); }
      }
      nc = block_sum_int(nc, sh.red_i);
      ncomp = block_sum_int(ncomp, sh.red_i);
      for (int ri = 0; ri < p.nrad; ++ri) {
        const int R = p.radii[ri];
        double m = -INFINITY, s = 0.0;
        int c = 0;
        for (int j = tid; j < M; j += kThreads) {
          double e = L.ell[j];
          if (e == -INFINITY) continue;
          int t = L.list[j];
          int dy = t / D2 - W, dx = t - (t / D2) * D2 - W;
          if (max(abs(dx), abs(dy)) > R) continue;
          lse_merge(m, s, e, 1.0);
          ++c;
        }
        c = block_sum_int(c, sh.red_i);
        block_lse(m, s, sh.red_m, sh.red_s);
        if (tid == 0) { sh.lse_m[ri] = m; sh.lse_s[ri] = s; sh.lse_c[ri] = c; }
      }
      if (tid == 0) {
        int layer = SKM_LAYER_IDL, ridx = p.nrad - 1, flags = relaxed_flag;
        bool want_hql = false;
        if (nc == 0) {
          layer = SKM_LAYER_BRL;
          flags |= SKM_FLAG_NO_CAND;
        } else if (p.mode == SKM_MODE_PLAIN) {
          ridx = p.nrad - 1;
        } else if (p.mode == SKM_MODE_FULL) {
          want_hql = true;
        } else {  // PROFILE, IDL, CNN without a network
          int acc = -1;
          for (int ri = 0; ri < p.nrad; ++ri) {
            if (sh.lse_c[ri] > 0) {
              double lnu = sh.lse_m[ri] + log(sh.lse_s[ri]);
              if (lnu >= p.log_tnu) { acc = ri; break; }
            }
          }
          if (acc >= 0) ridx = acc;
          else want_hql = p.mode != SKM_MODE_IDL;
        }
        if (want_hql) {
          if (ncomp >= max(2, p.min_hql)) layer = SKM_LAYER_HQL;
          else flags |= SKM_FLAG_NO_HQL;
        }
        sh.layer = layer; sh.radius_idx = ridx; sh.flags = flags;
        sh.n_cand = nc; sh.n_complete = ncomp;
        sh.lnu = nc > 0 ? sh.lse_m[ridx] + log(sh.lse_s[ridx]) : NAN;
      }
      __syncthreads();
    }
    const int layer = sh.layer;
    if (layer == SKM_LAYER_HQL) {
      // HQL runs in the dense-algebra kernels after this one
      if (tid == 0) {
        write_info(a, i, bx, by, SKM_LAYER_HQL, round, sh.n_cand, sh.n_complete, W, sh.flags,
                   phi, n0, sh.lnu);
        a.bstate[i] = kNeedHql + round;
      }
      __syncthreads();
      continue;
    }
    if (layer == SKM_LAYER_BRL) {
      for (int pix = tid; pix < B2; pix += kThreads) {
        int py = pix / B, px = pix - py * B;
        double v = fmin(fmax(floor(mean + 0.5), 0.0), 255.0);
        a.work[(size_t)(y0 + py) * p.stride + x0 + px] = (uint8_t)v;
        if (a.xhat && i < a.cap) a.xhat[(size_t)i * B2 + pix] = (float)mean;
      }
      if (tid == 0) {
        write_info(a, i, bx, by, SKM_LAYER_BRL, round, sh.n_cand, sh.n_complete, 0, sh.flags,
                   phi, n0, sh.lnu);
        a.bstate[i] = round;
      }
      __syncthreads();
      continue;
    }

    // 7. IDL: normalised weights over the accepted support area (eq. slpe)
    const int ridx = sh.radius_idx;
    const int R = p.radii[ridx];
    const double mstar = sh.lse_m[ridx];
    float* wv = reinterpret_cast<float*>(L.dval);
    double wsum = 0.0;
    for (int j = tid; j < M; j += kThreads) {
      double e = L.ell[j];
      float w = 0.f;
      if (e != -INFINITY) {
        int t = L.list[j];
        int dy = t / D2 - W, dx = t - (t / D2) * D2 - W;
        if (max(abs(dx), abs(dy)) <= R) w = expf((float)(e - mstar));
      }
      wv[j] = w;
      wsum += (double)w;
    }
    const double den = block_sum_double(wsum, sh.red_d);   // also a barrier

    // 8. weighted average of the prototypes, FP32 Kahan per pixel
    {
      const int G = kThreads / B2 > 0 ? kThreads / B2 : 1;
      const int g = tid / B2, pix = tid - g * B2;
      const int py = pix / B, px = pix - py * B;
      float acc = 0.f, comp = 0.f;
      if (g < G) {
        for (int j = g; j < M; j += G) {
          float w = wv[j];
          if (w == 0.f) continue;
          int t = L.list[j];
          int dy = t / D2 - W, dx = t - (t / D2) * D2 - W;
          float xv = (float)L.win[(W + r + dy + py) * Wd + (W + r + dx + px)];
          float y = w * xv - comp;
          float tt = acc + y;
          comp = (tt - acc) - y;
          acc = tt;
        }
      }
      __syncthreads();
      double* part = sh.part;
      if (g < G) part[tid] = (double)acc - (double)comp;
      __syncthreads();
      if (g == 0) {
        double tot = 0.0;
        for (int gg = 0; gg < G; ++gg) tot += part[gg * B2 + pix];
        double xh = tot / den;
        double v = fmin(fmax(floor(xh + 0.5), 0.0), 255.0);
        a.work[(size_t)(y0 + py) * p.stride + x0 + px] = (uint8_t)v;
        if (a.xhat && i < a.cap) a.xhat[(size_t)i * B2 + pix] = (float)xh;
      }
    }
    if (tid == 0) {
      write_info(a, i, bx, by, SKM_LAYER_IDL, round, sh.n_cand, sh.n_complete, R, sh.flags,
                 phi, n0, sh.lnu);
      a.bstate[i] = round;
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------- finalize
// blocks concealed in this round become received; count what is pending
__global__ __launch_bounds__(kThreads) void k_round_finalize(FrameArgs a, DevParams p) {
  __shared__ int s_pend;
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  const int n_lost = st->n_lost, round = st->round;
  if (threadIdx.x == 0) s_pend = 0;
  __syncthreads();
  const int B = p.B, B2 = B * B;
  for (int i = blockIdx.x; i < n_lost; i += gridDim.x) {
    int bs = a.bstate[i];
    if (bs >= kNeedHql && threadIdx.x == 0) atomicOr(&st->err, kErrHqlPending);
    if (bs == round) {
      int cell = a.blk[i];
      int by = cell / p.gw, bx = cell - by * p.gw;
      for (int pix = threadIdx.x; pix < B2; pix += blockDim.x) {
        int py = pix / B, px = pix - py * B;
        a.avail[(size_t)(by * B + py) * p.width + bx * B + px] = 1;
      }
    } else if (bs == 0 && threadIdx.x == 0) {
      ++s_pend;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_pend) atomicAdd(&st->remaining_acc, s_pend);
    __threadfence();
    int done = atomicAdd(&st->done_wgs, 1);
    if (done == (int)gridDim.x - 1) {
      __threadfence();
      int rem = atomicAdd(&st->remaining_acc, 0);
      st->remaining = rem;
      st->nq = 0;
      st->maxm0 = 0;
      st->round = round + 1;
      st->done_wgs = 0;
    }
  }
}

// ------------------------------------------------------------------- fill
// after the round limit: context mean (or frame mean) for pending blocks

__global__ void k_zero_fill(RoundState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { st->n_avail = 0; st->sum_avail = 0; }
}

__global__ __launch_bounds__(kThreads) void k_fill_stats(FrameArgs a, DevParams p) {
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  const long long npx = (long long)p.width * p.height;
  unsigned long long cnt = 0, sum = 0;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < npx;
       idx += (long long)gridDim.x * blockDim.x) {
    int y = (int)(idx / p.width), x = (int)(idx - (long long)y * p.width);
    if (a.avail[idx]) { ++cnt; sum += a.work[(size_t)y * p.stride + x]; }
  }
  cnt = wave_sum(cnt);
  sum = wave_sum(sum);
  if (lane_id() == 0 && cnt) {
    atomicAdd(&st->n_avail, cnt);
    atomicAdd(&st->sum_avail, sum);
  }
}

__global__ __launch_bounds__(kThreads) void k_fill(FrameArgs a, DevParams p) {
  __shared__ int s_red[4];
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  const int n_lost = st->n_lost, round = st->round;
  const int B = p.B, B2 = B * B, F = p.F, r = p.r;
  const double fmean = st->n_avail ? (double)st->sum_avail / (double)st->n_avail : 0.0;
  for (int i = blockIdx.x; i < n_lost; i += gridDim.x) {
    if (a.bstate[i] != 0) continue;
    int cell = a.blk[i];
    int by = cell / p.gw, bx = cell - by * p.gw;
    int xr = bx * B - r, yr = by * B - r;
    int c = 0, s = 0;
    for (int pos = threadIdx.x; pos < F * F; pos += blockDim.x) {
      int fy = pos / F, fx = pos - fy * F;
      bool ring = fy < r || fy >= r + B || fx < r || fx >= r + B;
      int gy = yr + fy, gx = xr + fx;
      if (ring && gy >= 0 && gy < p.height && gx >= 0 && gx < p.width &&
          a.avail[(size_t)gy * p.width + gx]) {
        ++c;
        s += a.work[(size_t)gy * p.stride + gx];
      }
    }
    c = block_sum_int(c, s_red);
    s = block_sum_int(s, s_red);
    double v = c > 0 ? (double)s / (double)c : fmean;
    for (int pix = threadIdx.x; pix < B2; pix += blockDim.x) {
      int py = pix / B, px = pix - py * B;
      a.work[(size_t)(by * B + py) * p.stride + bx * B + px] =
          (uint8_t)fmin(fmax(floor(v + 0.5), 0.0), 255.0);
      if (a.xhat && i < a.cap) a.xhat[(size_t)i * B2 + pix] = (float)v;
    }
    if (threadIdx.x == 0) {
      write_info(a, i, bx, by, SKM_LAYER_FILL, round, -1, -1, 0,
                 c > 0 ? 0 : SKM_FLAG_EMPTY_CTX, 0, c, NAN);
      a.bstate[i] = round;
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------- launchers

static int grid_for(long long work, int per) {
  long long g = (work + per - 1) / per;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

hipError_t launch_init(const FrameArgs& a, const DevParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, s, a.st);
  hipLaunchKernelGGL(k_init, dim3(grid_for((long long)p.width * p.height, kThreads * 8)),
                     dim3(kThreads), 0, s, a, p);
  int ncell = p.gh * p.gw;
  hipLaunchKernelGGL(k_cells, dim3(grid_for(ncell, kThreads)), dim3(kThreads), 0, s, a, p);
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, a, p);
  return hipGetLastError();
}

hipError_t launch_main(const FrameArgs& a, const DevParams& p, int max_blocks, int dist_only,
                       hipStream_t s) {
  size_t lds = main_lds_bytes(p);
  int g = max_blocks < 1 ? 1 : (max_blocks > 2048 ? 2048 : max_blocks);
  hipLaunchKernelGGL(k_round_main, dim3(g), dim3(kThreads), lds, s, a, p, dist_only);
  return hipGetLastError();
}

hipError_t launch_prep(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s) {
  int gw = grid_for(max_blocks, kThreads / 64);
  hipLaunchKernelGGL(k_round_prep, dim3(gw), dim3(kThreads), 0, s, a, p);
  return hipGetLastError();
}

hipError_t launch_est(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s) {
  return launch_main(a, p, max_blocks, 0, s);
}

hipError_t launch_finalize(const FrameArgs& a, const DevParams& p, int max_blocks,
                           hipStream_t s) {
  int gf = max_blocks < 1 ? 1 : (max_blocks > 1024 ? 1024 : max_blocks);
  hipLaunchKernelGGL(k_round_finalize, dim3(gf), dim3(kThreads), 0, s, a, p);
  return hipGetLastError();
}

hipError_t launch_dist(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s) {
  return launch_main(a, p, max_blocks, 1, s);
}

hipError_t launch_fill(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_fill, dim3(1), dim3(64), 0, s, a.st);
  hipLaunchKernelGGL(k_fill_stats, dim3(grid_for((long long)p.width * p.height, kThreads * 8)),
                     dim3(kThreads), 0, s, a, p);
  int g = max_blocks < 1 ? 1 : (max_blocks > 2048 ? 2048 : max_blocks);
  hipLaunchKernelGGL(k_fill, dim3(g), dim3(kThreads), 0, s, a, p);
  return hipGetLastError();
}

hipError_t set_main_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_round_main,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace skm
