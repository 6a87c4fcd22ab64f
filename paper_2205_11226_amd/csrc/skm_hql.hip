// High quality layer (HQL): full K-MMSE for one lost block per workgroup.
//
// Paper (Koloda et al., arXiv 2205.11226), Sec. "K-MMSE overview":
//   x0_hat = x~0(beta) + alpha C_XY C_YY^-1 (y0 - y~0(beta))          (eq. kmmse,
//            with H = covariance-submatrix scaling, eq. bandwidthScaled)
//   weights exp(-(y0-y_j)^T (beta C_YY)^-1 (y0-y_j) / 2), normalised   (eq. weights)
//   beta = argmin ||y0 - sum_j w_j(beta) y_j||^2                       (eq. epsy)
//   alpha = argmin (1/|I0|) sum_{i in I0} ||x_i - x_i_hat||^2,
//           I0 = the N_y + 1 observations closest to y0                (eq. epsx)
// Readings where the paper is silent: C_ZZ normalised by 1/M with a ridge
// lambda = ridge_rel tr(C_YY)/N_y + 1e-12 on C_YY; beta from the first
// minimiser of a grid D0 2^(g/2), g = -8..24 (grid values within a relative
// 1e-12 of the smallest count as minimisers), refined by 40 golden-section
// steps on log beta and kept only if better by that margin; I0 by Euclidean distance with
// ties to the lower raster index; each x_i predicted leave-one-out; alpha in
// closed form (x_i_hat is affine in alpha).
//
// The candidate set is every admissible candidate whose ring covers all of
// the block's known context pixels.  All algebra is FP64; the covariance
// comes from an exact integer Gram (v_dot4_u32_u8 on the 8-bit pixels).
// Scratch: one global slot per workgroup (layout in hql_layout).
#include "skm_device.h"

namespace skm {

struct HqlLayout {
  size_t yt, xt, cyy, axy, v, v0, y0, meany, meanx, dm0, ytil, xtil, vn, dch, zch, i0;
  // partly known contexts (hql_partial): availability bytes, overlap counts,
  // integer Grams of the masks (gn), of values by masks (gs, gsx), and a copy
  // of C_YY for the repair's retries
  size_t ot, cn, gn, gs, gsx, cyy0;
  size_t total;
  int ldm;     // leading dimension (candidates) of yt / xt, multiple of 64
  int ldz;     // row length of zch: B^2 + NY
  int ny;      // NY: most context pixels of a block (ring, and own pixels when received)
};

__host__ __device__ inline HqlLayout hql_layout(const DevParams& p) {
  HqlLayout h;
  const size_t MC = p.MC, B2 = (size_t)p.B * p.B;
  const size_t NY = (size_t)p.NR + B2;          // a block's received own pixels join y0
  h.ny = (int)NY;
  h.ldm = (int)align_up(MC, 64);
  h.ldz = (int)(B2 + NY);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
  h.yt = take(NY * h.ldm);
  h.xt = take(B2 * h.ldm);
  h.cyy = take(8 * NY * NY);
  h.axy = take(8 * B2 * NY);
  h.v = take(8 * MC * NY);
  h.v0 = take(8 * NY);
  h.y0 = take(8 * NY);
  h.meany = take(8 * NY);
  h.meanx = take(8 * B2);
  h.dm0 = take(8 * MC);
  h.ytil = take(8 * NY);
  h.xtil = take(8 * B2);
  h.vn = take(8 * MC);
  h.dch = take(8 * 64 * MC);
  h.zch = take(8 * 64 * (B2 + NY));
  h.i0 = take(4 * MC);
  const bool pt = p.hql_partial != 0;
  h.ot = take(pt ? NY * h.ldm : 0);
  h.cn = take(pt ? 4 * MC : 0);
  h.gn = take(pt ? 4 * NY * NY : 0);
  h.gs = take(pt ? 4 * NY * NY : 0);
  h.gsx = take(pt ? 4 * B2 * NY : 0);
  h.cyy0 = take(pt ? 8 * NY * NY : 0);
  h.total = o;
  return h;
}

size_t hql_slot_bytes(const DevParams& p) { return hql_layout(p).total; }

int hql_slots(const DevParams& p) {
  const size_t n = kHqlScratchBudget / hql_slot_bytes(p);
  return n < (size_t)kHqlSlots ? kHqlSlots : (n > (size_t)kHqlSlotsMax ? kHqlSlotsMax : (int)n);
}

// the estimation kernel's layout, with the window region large enough for
// the HQL tiles that reuse it
size_t hql_lds_bytes(const DevParams& p) {
  size_t offs[10];
  main_lds_layout(p, offs);
  size_t need = (size_t)4 * p.Wd * p.Wd;
  need = need > 16384 ? need : 16384;                      // FP64 GEMM tiles
  need = need > 2 * 16 * 65 * 8 ? need : 2 * 16 * 65 * 8;   // (pitch 65 for the sums)
  need = need > (size_t)2 * 64 * 17 * 4 ? need : (size_t)2 * 64 * 17 * 4;   // Gram tiles
  const size_t ny = (size_t)p.NR + (size_t)p.B * p.B;
  need = need > 8 * ny ? need : 8 * ny;                     // Cholesky pivot row
  return align_up(offs[9] + need, 16);
}

// PSD repair of a pairwise-complete C_YY: lambda x 10, at most this often
constexpr int kPsdRepair = 6;
__device__ __constant__ const double kPow10[kPsdRepair + 1] = {1.0, 10.0, 100.0, 1e3, 1e4, 1e5,
                                                                1e6};

// eps_y values within this relative margin count as equal: where eps_y is
// flat (as beta -> 0 the weights become one-hot on the nearest candidate), the
// argmin of eq. epsy is not unique, so the smallest flat beta is taken and a
// refined beta must improve on it by more than the margin
constexpr double kEpsTieRel = 1e-12;

struct HqlShared {
  double red[kThreads / 64];
  double eg[33];                 // eps_y on the beta grid g = -8 .. 24
  double dk, lam, S, eps, dmin;
  int fail;
  double rowS[64];
};

// deterministic workgroup sum (fixed shuffle tree, fixed wave order)
static __device__ __forceinline__ double block_sum_d(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

static __device__ __forceinline__ double block_min_d(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  return fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// Covariance block from the exact integer Gram of two u8 row sets:
// out[i*ldo + j] = (sum_k P[i][k] Q[j][k]) / M - mp[i] mq[j].  Rows have
// leading dimension ld (zero padded beyond M, multiple of 64).  64x64
// output tiles, K staged 64 bytes at a time in LDS, 4x4 per thread,
// v_dot4_u32_u8.  With sym (P == Q), only the lower tiles are computed and
// mirrored.
static __device__ void gram_cov(const uint8_t* P, const uint8_t* Q, int R1, int R2, int ld, int M,
                                double* out, int ldo, const double* mp, const double* mq, bool sym,
                                uint32_t* ta, uint32_t* tb) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const int nt1 = (R1 + 63) / 64, nt2 = (R2 + 63) / 64;
  const double invM = 1.0 / (double)M;
  for (int t1 = 0; t1 < nt1; ++t1) {
    for (int t2 = 0; t2 < nt2; ++t2) {
      if (sym && t2 > t1) continue;
      uint32_t acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0u;
      for (int kk = 0; kk < ld; kk += 64) {
        // stage 64 rows x 16 words of each operand (row pitch 17 words)
        for (int e = tid; e < 64 * 16; e += kThreads) {
          const int row = e >> 4, w = e & 15;
          const int r1 = t1 * 64 + row, r2 = t2 * 64 + row;
          ta[row * 17 + w] = r1 < R1 ? *(const uint32_t*)(P + (size_t)r1 * ld + kk + 4 * w) : 0u;
          tb[row * 17 + w] = r2 < R2 ? *(const uint32_t*)(Q + (size_t)r2 * ld + kk + 4 * w) : 0u;
        }
        __syncthreads();
#pragma unroll 4
        for (int w = 0; w < 16; ++w) {
          uint32_t av[4], bv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) av[a] = ta[(ty * 4 + a) * 17 + w];
#pragma unroll
          for (int b = 0; b < 4; ++b) bv[b] = tb[(tx * 4 + b) * 17 + w];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_udot4(av[a], bv[b], acc[a][b], false);
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = t1 * 64 + ty * 4 + a, j = t2 * 64 + tx * 4 + b;
          if (i < R1 && j < R2) {
            const double c = (double)acc[a][b] * invM - mp[i] * mq[j];
            out[(size_t)i * ldo + j] = c;
            if (sym) out[(size_t)j * ldo + i] = c;
          }
        }
      }
    }
  }
  __syncthreads();
}

// Exact integer Gram P Q^T (rows of P and Q are R1 and R2 byte vectors of
// length ld, zero padded) stored as Out, without normalisation: the tiles of
// gram_cov.
template <typename Out>
static __device__ void gram_raw(const uint8_t* P, const uint8_t* Q, int R1, int R2, int ld,
                                Out* out, int ldo, bool sym, uint32_t* ta, uint32_t* tb) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const int nt1 = (R1 + 63) / 64, nt2 = (R2 + 63) / 64;
  for (int t1 = 0; t1 < nt1; ++t1) {
    for (int t2 = 0; t2 < nt2; ++t2) {
      if (sym && t2 > t1) continue;
      uint32_t acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0u;
      for (int kk = 0; kk < ld; kk += 64) {
        for (int e = tid; e < 64 * 16; e += kThreads) {
          const int row = e >> 4, w = e & 15;
          const int r1 = t1 * 64 + row, r2 = t2 * 64 + row;
          ta[row * 17 + w] = r1 < R1 ? *(const uint32_t*)(P + (size_t)r1 * ld + kk + 4 * w) : 0u;
          tb[row * 17 + w] = r2 < R2 ? *(const uint32_t*)(Q + (size_t)r2 * ld + kk + 4 * w) : 0u;
        }
        __syncthreads();
#pragma unroll 4
        for (int w = 0; w < 16; ++w) {
          uint32_t av[4], bv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) av[a] = ta[(ty * 4 + a) * 17 + w];
#pragma unroll
          for (int b = 0; b < 4; ++b) bv[b] = tb[(tx * 4 + b) * 17 + w];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_udot4(av[a], bv[b], acc[a][b], false);
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = t1 * 64 + ty * 4 + a, j = t2 * 64 + tx * 4 + b;
          if (i < R1 && j < R2) {
            out[(size_t)i * ldo + j] = (Out)acc[a][b];
            if (sym) out[(size_t)j * ldo + i] = (Out)acc[a][b];
          }
        }
      }
    }
  }
  __syncthreads();
}

// One evaluation of eps_y(beta) (eq. epsy): weights e_j = exp(-dm0_j/(2 beta)
// - max), S = sum e_j, y~ = sum e_j y_j / S; returns ||y0 - y~||^2.  Leaves
// ew, S (in hs.S) and ytil for the caller.  With xt != nullptr also x~.
static __device__ double eval_eps(double beta, int Mc, int Ny, int B2, int ldm, const double* dm0,
                                  double dmin, double* ew, const uint8_t* yt, const uint8_t* xt,
                                  const double* y0, double* ytil, double* xtil, HqlShared& hs) {
  const int tid = threadIdx.x;
  const double inv2b = 1.0 / (2.0 * beta);      // one division per evaluation
  const double m = -dmin * inv2b;
  double s = 0.0;
  for (int j = tid; j < Mc; j += kThreads) {
    const double e = exp(-dm0[j] * inv2b - m);
    ew[j] = e;
    s += e;
  }
  const double S = block_sum_d(s, hs.red);     // barrier: ew visible
  // eight rows per wave at a time; a lane takes four consecutive candidates
  // per step (one 32-bit load per row: the byte rows are zero-padded to ldm,
  // a multiple of 64), then fixed-order wave sums
  const int lane = lane_id(), wave = wave_id();
  double part = 0.0;
  auto rows8 = [&](const uint8_t* base, int a0, int nrow, double* acc) {
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = 0.0;
    for (int j = 4 * lane; j < Mc; j += 256) {
      double e[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) e[q] = j + q < Mc ? ew[j + q] : 0.0;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        if (a0 + r < nrow) {
          const uint32_t w = *reinterpret_cast<const uint32_t*>(base + (size_t)(a0 + r) * ldm + j);
          acc[r] += e[0] * (double)(w & 0xffu) + e[1] * (double)((w >> 8) & 0xffu) +
                    e[2] * (double)((w >> 16) & 0xffu) + e[3] * (double)(w >> 24);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = wave_sum(acc[r]);
  };
  for (int a0 = 8 * wave; a0 < Ny; a0 += 8 * (kThreads / 64)) {
    double acc[8];
    rows8(yt, a0, Ny, acc);
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        if (a0 + r < Ny) {
          const double yt_a = acc[r] / S;
          ytil[a0 + r] = yt_a;
          const double d = y0[a0 + r] - yt_a;
          part += d * d;
        }
      }
    }
  }
  if (xt) {
    for (int q0 = 8 * wave; q0 < B2; q0 += 8 * (kThreads / 64)) {
      double acc[8];
      rows8(xt, q0, B2, acc);
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
          if (q0 + r < B2) xtil[q0 + r] = acc[r] / S;
      }
    }
  }
  hs.S = S;
  return block_sum_d(part, hs.red);
}

// The HQL blocks h = blockIdx.x, blockIdx.x + gridDim.x, ... of one frame's
// list (n_hql entries).  `first` is true until the workgroup has taken a
// block (from any frame).
static __device__ __forceinline__ void hql_frame(const FrameArgs& a, const DevParams& p,
                                                 unsigned char* ws, size_t slot_bytes, int round,
                                                 int n_hql, bool& first, unsigned char* lds_raw,
                                                 BlockShared& sh, HqlShared& hs, int* pend) {
  const MainLds L = carve_main_lds(lds_raw, p);
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int B = p.B, r = p.r, W = p.W, Wd = p.Wd;
  const int B2 = B * B;
  const int qbase = W * Wd + W;
  phase_tables(p, L, sh);
  const int NU = sh.NU;

  const HqlLayout hl = hql_layout(p);
  unsigned char* slot = ws + (size_t)blockIdx.x * slot_bytes;
  uint8_t* yt = slot + hl.yt;
  uint8_t* xt = slot + hl.xt;
  double* cyy = (double*)(slot + hl.cyy);
  double* axy = (double*)(slot + hl.axy);
  double* V = (double*)(slot + hl.v);
  double* v0 = (double*)(slot + hl.v0);
  double* y0v = (double*)(slot + hl.y0);
  double* meany = (double*)(slot + hl.meany);
  double* meanx = (double*)(slot + hl.meanx);
  double* dm0 = (double*)(slot + hl.dm0);
  // the candidates' weights of the eps_y evaluations live in LDS (the log
  // weight array is free once the complete candidates are listed)
  double* ew = L.ell;
  double* ytil = (double*)(slot + hl.ytil);
  double* xtil = (double*)(slot + hl.xtil);
  double* vn = (double*)(slot + hl.vn);
  double* dch = (double*)(slot + hl.dch);
  double* zch = (double*)(slot + hl.zch);
  int* i0l = (int*)(slot + hl.i0);
  const bool hp = p.hql_partial != 0;                 // partly known contexts (see hql_layout)
  uint8_t* ot = slot + hl.ot;
  int* cnl = (int*)(slot + hl.cn);
  int* gn = (int*)(slot + hl.gn);
  int* gs = (int*)(slot + hl.gs);
  int* gsx = (int*)(slot + hl.gsx);
  double* cyy0 = (double*)(slot + hl.cyy0);
  const int ldm = hl.ldm, ldz = hl.ldz, NRs = hl.ny;      // NRs: row stride of Ny rows

  // LDS reuse once the window has been gathered
  uint32_t* ta = (uint32_t*)L.winp;                  // gram tiles, 2 x 64 x 17 words
  uint32_t* tb = ta + 64 * 17;
  double* piv = (double*)L.winp;                     // Cholesky pivot row
  double* ga = (double*)L.winp;                      // FP64 GEMM tiles, 2 x 16 x 64
  double* gb = ga + 16 * 64;
  double* ca = ga;                                   // leave-one-out sums: 2 x 16 x 64,
  double* cb = ga + 16 * 65;                         //   row pitch 65
  uint16_t* m0off = (uint16_t*)L.qu;                 // known ring pixels (footprint offsets)
  uint16_t* compo = L.selo;                          // complete candidates: window offset
  int* compd = (int*)L.selw;                         //   and exact Euclidean distance

  for (int h = blockIdx.x; h < n_hql; h += gridDim.x) {
    const int i = a.hql_list[h];
    const int cell = a.blk[i];
    const int by = cell / p.gw, bx = cell - by * p.gw;
    const int x0 = bx * B, y0 = by * B;

    // -- candidates: the estimation kernel's phases, then the complete ones.
    //    Staging ORs the window's availability into rowbits, so a workgroup
    //    that takes several blocks clears it for each one.
    if (!first) {
      for (int k = tid; k < 2 * Wd; k += kThreads) L.rowbits[k] = 0ull;
      __syncthreads();
    }
    first = false;
    phase_stage(a, p, L, x0 - r - W, y0 - r - W);
    // context units: the ring, then the block's own pixel pairs if it holds
    // received pixels
    const bool partial = (a.m0cnt[i] & kPartialBit) != 0;
    const int NUe = partial ? NU + B2 / 2 : NU;
    const RingStats rs = phase_context(p, L, sh, NU, NUe);
    const int n0 = rs.n0;
    const int M = phase_candidates(p, L, sh);
    const int nmin = max(1, (p.min_pct * n0 + 99) / 100);
    {
      const int per = (M + kThreads - 1) / kThreads;
      const int j0 = min(M, tid * per), j1 = min(M, j0 + per);
      int cnt = 0;
      for (int j = j0; j < j1; ++j) {
        int d, n;
        cand_distance(L, cand_off(L.cand[j]), NUe, d, n);
        // HQL's candidates: complete contexts, or (hql_partial) every
        // admissible one, its overlap count kept for the I0 order
        const bool comp = (hp || n == n0) && n >= nmin;
        L.ell[j] = comp ? (double)d : -1.0;
        if (hp) L.cand[j] = (L.cand[j] & 0x3ffffu) | ((uint32_t)n << 18);
        cnt += comp;
      }
      int tot = 0;
      int pos = block_excl_scan(cnt, sh.scan, &tot);
      for (int j = j0; j < j1; ++j) {
        if (L.ell[j] >= 0.0) {
          compo[pos] = (uint16_t)cand_off(L.cand[j]);
          compd[pos] = (int)L.ell[j];
          if (hp) cnl[pos] = cand_n(L.cand[j]);
          ++pos;
        }
      }
      if (tid == 0) sh.M = tot;
    }
    // known context pixels in unit order (ring pairs in raster order, then
    // the block's own pairs)
    {
      const int per = (NUe + kThreads - 1) / kThreads;
      const int u0 = min(NUe, tid * per), u1 = min(NUe, u0 + per);
      int cnt = 0;
      for (int u = u0; u < u1; ++u) {
        const uint32_t qp = L.qu[u].x;
        cnt += ((int16_t)(qp & 0xffffu) >= 0) + ((int16_t)(qp >> 16) >= 0);
      }
      int tot = 0;
      int pos = block_excl_scan(cnt, sh.scan, &tot);
      uint16_t tmp[2 * 4];
      int nt = 0;
      // read all owned units before writing: m0off aliases the unit array
      for (int u = u0; u < u1 && nt < 8; ++u) {
        const uint2 q = L.qu[u];
        if ((int16_t)(q.x & 0xffffu) >= 0) tmp[nt++] = (uint16_t)q.y;
        if ((int16_t)(q.x >> 16) >= 0) tmp[nt++] = (uint16_t)(q.y + 1);
      }
      __syncthreads();
      for (int t = 0; t < nt; ++t) m0off[pos + t] = tmp[t];
    }
    __syncthreads();
    const int Mc = sh.M, Ny = n0;

    // -- gather Y (Ny x Mc), X (B2 x Mc) as bytes, zero padded to ldm; y0.
    //    Unknown context pixels of a candidate (hql_partial) read 0, with
    //    availability 0 in ot.
    for (int aa = wave; aa < Ny; aa += kThreads / 64) {
      const int off = m0off[aa];
      for (int k = lane; k < ldm; k += 64) {
        const int v = k < Mc ? (int)(int16_t)(L.winp[compo[k] + off] & 0xffffu) : -1;
        yt[(size_t)aa * ldm + k] = v >= 0 ? (uint8_t)v : (uint8_t)0;
        if (hp) ot[(size_t)aa * ldm + k] = v >= 0 ? (uint8_t)1 : (uint8_t)0;
      }
    }
    for (int q = wave; q < B2; q += kThreads / 64) {
      const int off = (r + q / B) * Wd + r + (q % B);
      for (int k = lane; k < ldm; k += 64)
        xt[(size_t)q * ldm + k] = k < Mc ? (uint8_t)(L.winp[compo[k] + off] & 0xffu) : (uint8_t)0;
    }
    for (int aa = tid; aa < Ny; aa += kThreads)
      y0v[aa] = (double)(int)(int16_t)(L.winp[qbase + m0off[aa]] & 0xffffu);
    __syncthreads();
    if (!hp) {
      // column means: a wave per row, exact integer sums
      for (int aa = wave; aa < Ny; aa += kThreads / 64) {
        int s = 0;
        for (int k = lane; k < Mc; k += 64) s += yt[(size_t)aa * ldm + k];
        s = wave_sum(s);
        if (lane == 0) meany[aa] = (double)s / (double)Mc;
      }
      for (int q = wave; q < B2; q += kThreads / 64) {
        int s = 0;
        for (int k = lane; k < Mc; k += 64) s += xt[(size_t)q * ldm + k];
        s = wave_sum(s);
        if (lane == 0) meanx[q] = (double)s / (double)Mc;
      }
      __syncthreads();

      // -- covariance blocks C_YY (Ny x Ny) and C_XY (B2 x Ny), 1/M normalised
      gram_cov(yt, yt, Ny, Ny, ldm, Mc, cyy, NRs, meany, meany, true, ta, tb);
      gram_cov(xt, yt, B2, Ny, ldm, Mc, axy, NRs, meanx, meany, false, ta, tb);
    } else {
      // -- pairwise-complete covariance: for coordinates a, b the candidates
      //    knowing both (N_ab of them); exact integer Grams of the values
      //    (unknown = 0) and of the availability, then
      //    C_ab = G_ab / N_ab - S_a(b) S_b(a) / N_ab^2 with S_a(b) the sum of
      //    coordinate a over those candidates (0 where N_ab = 0).  The x
      //    coordinates are always known: N_qb = N_bb.
      gram_raw(yt, yt, Ny, Ny, ldm, cyy, NRs, true, ta, tb);
      gram_raw(ot, ot, Ny, Ny, ldm, gn, Ny, true, ta, tb);
      gram_raw(yt, ot, Ny, Ny, ldm, gs, Ny, false, ta, tb);
      gram_raw(xt, yt, B2, Ny, ldm, axy, NRs, false, ta, tb);
      gram_raw(xt, ot, B2, Ny, ldm, gsx, Ny, false, ta, tb);
      for (int e = tid; e < Ny * Ny; e += kThreads) {
        const int aa = e / Ny, bb = e - aa * Ny;
        const double n = (double)gn[e];
        double* c = cyy + (size_t)aa * NRs + bb;
        const double v = n > 0.0 ? *c / n - ((double)gs[e] * (double)gs[bb * Ny + aa]) / (n * n)
                                 : 0.0;
        *c = v;
        cyy0[e] = v;
      }
      for (int e = tid; e < B2 * Ny; e += kThreads) {
        const int q = e / Ny, bb = e - q * Ny;
        const double n = (double)gn[bb * Ny + bb];
        double* c = axy + (size_t)q * NRs + bb;
        *c = n > 0.0 ? *c / n - ((double)gsx[e] / n) * ((double)gs[bb * Ny + bb] / n) : 0.0;
      }
      __syncthreads();
      // -- unknown context pixels of a candidate: the coordinate's mean over
      //    the candidates knowing it, rounded half up (y0's pixel if none)
      for (int aa = wave; aa < Ny; aa += kThreads / 64) {
        const int n = gn[aa * Ny + aa], sm = gs[aa * Ny + aa];
        const int fill = n > 0 ? (2 * sm + n) / (2 * n) : (int)y0v[aa];
        for (int k = lane; k < Mc; k += 64)
          if (!ot[(size_t)aa * ldm + k]) yt[(size_t)aa * ldm + k] = (uint8_t)fill;
      }
      __syncthreads();
    }

    // -- ridge and Cholesky C_YY = L L^T (left-looking, in place, lower).
    //    A pairwise-complete C_YY (hql_partial) need not be positive
    //    semi-definite: while a pivot is <= 0 the factorisation restarts
    //    from the saved C_YY with lambda ten times larger, at most
    //    kPsdRepair times.
    double lam0;
    {
      double tr = 0.0;
      for (int aa = tid; aa < Ny; aa += kThreads) tr += cyy[(size_t)aa * NRs + aa];
      tr = block_sum_d(tr, hs.red);
      lam0 = p.ridge_rel * tr / (double)Ny + 1e-12;
    }
    for (int rep = 0; rep <= (hp ? kPsdRepair : 0); ++rep) {
      if (rep > 0) {
        __syncthreads();
        for (int e = tid; e < Ny * Ny; e += kThreads) {
          const int aa = e / Ny, bb = e - aa * Ny;
          cyy[(size_t)aa * NRs + bb] = cyy0[e];
        }
        __syncthreads();
      }
      const double lam = lam0 * kPow10[rep];
      for (int aa = tid; aa < Ny; aa += kThreads) cyy[(size_t)aa * NRs + aa] += lam;
      if (tid == 0) hs.fail = 0;
      __syncthreads();
      for (int k = 0; k < Ny; ++k) {
        const double* rowk = cyy + (size_t)k * NRs;
        for (int m = tid; m < k; m += kThreads) piv[m] = rowk[m];
        if (wave == 0) {
          double s = 0.0;
          for (int m = lane; m < k; m += 64) s += rowk[m] * rowk[m];
          s = wave_sum(s);
          if (lane == 0) {
            const double dd = rowk[k] - s;
            if (!(dd > 0.0)) hs.fail = 1;
            hs.dk = dd > 0.0 ? sqrt(dd) : 1.0;
            cyy[(size_t)k * NRs + k] = hs.dk;
          }
        }
        __syncthreads();
        if (hs.fail) break;                 // uniform: written before the barrier
        const double dk = hs.dk;
        for (int ii = k + 1 + tid; ii < Ny; ii += kThreads) {
          double* rowi = cyy + (size_t)ii * NRs;
          double s = rowi[k];
          for (int m = 0; m < k; ++m) s -= rowi[m] * piv[m];
          rowi[k] = s / dk;
        }
        __syncthreads();
      }
      if (!hs.fail) break;
    }
    if (hs.fail) {
      // C_YY + lambda I is not positive definite in FP64 (a pivot <= 0): the
      // covariance model of eq. kmmse does not exist for this block, which
      // takes the context mean of eq. mean, flagged
      const double mean = (double)rs.sum / (double)n0;
      const uint8_t u8 = (uint8_t)fmin(fmax(floor(mean + 0.5), 0.0), 255.0);
      for (int q = tid; q < B2; q += kThreads) {
        const int py = q / B, px = q - py * B;
        if (!partial || a.val[(size_t)(y0 + py) * p.width + x0 + px] < 0)
          a.work[(size_t)(y0 + py) * p.stride + x0 + px] = u8;
        if (a.xhat && i < a.cap) a.xhat[(size_t)i * B2 + q] = (float)mean;
      }
      if (tid == 0) {
        if (a.info && i < a.cap) {
          a.info[i].layer = SKM_LAYER_BRL;
          a.info[i].flags |= SKM_FLAG_HQL_SINGULAR;
        }
        a.bstate[i] = round;
        if (pend) atomicSub(pend, 1);
      }
      __syncthreads();
      continue;
    }
    const double* Lc = cyy;   // lower triangle holds L

    // -- A = C_XY C_YY^-1: row q of C_XY solves L L^T a^T = c^T (in place)
    for (int q = tid; q < B2; q += kThreads) {
      double* row = axy + (size_t)q * NRs;
      for (int k = 0; k < Ny; ++k) {
        const double* lk = Lc + (size_t)k * NRs;
        double s = row[k];
        for (int m = 0; m < k; ++m) s -= lk[m] * row[m];
        row[k] = s / lk[k];
      }
      for (int k = Ny - 1; k >= 0; --k) {
        double s = row[k];
        for (int m = k + 1; m < Ny; ++m) s -= Lc[(size_t)m * NRs + k] * row[m];
        row[k] = s / Lc[(size_t)k * NRs + k];
      }
    }
    // -- whitening: V[j] = L^-1 y_j for every candidate, v0 = L^-1 y0
    for (int j = tid; j <= Mc; j += kThreads) {
      double* row = j < Mc ? V + (size_t)j * NRs : v0;
      for (int k = 0; k < Ny; ++k) {
        const double* lk = Lc + (size_t)k * NRs;
        double s = j < Mc ? (double)yt[(size_t)k * ldm + j] : y0v[k];
        for (int m = 0; m < k; ++m) s -= lk[m] * row[m];
        row[k] = s / lk[k];
      }
    }
    __syncthreads();
    // Mahalanobis distances to y0 and squared norms of the whitened candidates
    double dmin = INFINITY;
    for (int j = tid; j < Mc; j += kThreads) {
      const double* row = V + (size_t)j * NRs;
      double s = 0.0, nn = 0.0;
      for (int k = 0; k < Ny; ++k) {
        const double d = row[k] - v0[k];
        s += d * d;
        nn += row[k] * row[k];
      }
      dm0[j] = s;
      vn[j] = nn;
      dmin = fmin(dmin, s);
    }
    dmin = block_min_d(dmin, hs.red);

    // -- beta: first grid minimiser, golden-section refinement on log beta
    const double D0 = fmax(dmin, 1e-9);
    double emin = INFINITY;
    for (int g = -8; g <= 24; ++g) {
      const double bt = D0 * exp2((double)g / 2.0);
      const double e = eval_eps(bt, Mc, Ny, B2, ldm, dm0, dmin, ew, yt, nullptr, y0v, ytil, nullptr, hs);
      if (tid == 0) hs.eg[g + 8] = e;
      emin = fmin(emin, e);
    }
    __syncthreads();
    int gstar = 24;
    for (int g = 24; g >= -8; --g)
      if (hs.eg[g + 8] <= emin * (1.0 + kEpsTieRel)) gstar = g;
    const double best_eps = hs.eg[gstar + 8];
    double beta;
    {
      const int glo = max(gstar - 1, -8), ghi = min(gstar + 1, 24);
      double at = log(D0 * exp2((double)glo / 2.0));
      double bt = log(D0 * exp2((double)ghi / 2.0));
      const double invphi = (sqrt(5.0) - 1.0) / 2.0;
      double ct = bt - invphi * (bt - at);
      double dt = at + invphi * (bt - at);
      double fc = eval_eps(exp(ct), Mc, Ny, B2, ldm, dm0, dmin, ew, yt, nullptr, y0v, ytil, nullptr, hs);
      double fd = eval_eps(exp(dt), Mc, Ny, B2, ldm, dm0, dmin, ew, yt, nullptr, y0v, ytil, nullptr, hs);
      for (int it = 0; it < 40; ++it) {
        if (fc <= fd) {
          bt = dt; dt = ct; fd = fc;
          ct = bt - invphi * (bt - at);
          fc = eval_eps(exp(ct), Mc, Ny, B2, ldm, dm0, dmin, ew, yt, nullptr, y0v, ytil, nullptr, hs);
        } else {
          at = ct; ct = dt; fc = fd;
          dt = at + invphi * (bt - at);
          fd = eval_eps(exp(dt), Mc, Ny, B2, ldm, dm0, dmin, ew, yt, nullptr, y0v, ytil, nullptr, hs);
        }
      }
      beta = exp(0.5 * (at + bt));
      const double eb = eval_eps(beta, Mc, Ny, B2, ldm, dm0, dmin, ew, yt, nullptr, y0v, ytil, nullptr, hs);
      if (!(eb < best_eps * (1.0 - kEpsTieRel))) beta = D0 * exp2((double)gstar / 2.0);
    }

    // -- I0: the min(Ny + 1, Mc) candidates of smallest (distance, index),
    //    found by bisection on the packed key; listed in candidate order
    //    (hql_partial: of smallest d / n, as floor(d 2^20 / n), which keeps
    //    the order of the fractions: distinct ones differ by >= 2^20 / n^2 > 3)
    const int k0 = min(Ny + 1, Mc);
    {
      auto key = [&](int j) -> long long {
        const long long d = compd[j];
        return (hp ? (d << 20) / cnl[j] : d) << 13 | j;
      };
      long long lo = 0, hi = hp ? (1ll << 60) - 1 : (1ll << 40) - 1;
      while (lo < hi) {
        const long long mid = lo + ((hi - lo) >> 1);
        int c = 0;
        for (int j = tid; j < Mc; j += kThreads) c += key(j) <= mid;
        c = (int)block_sum_d((double)c, hs.red);
        if (c >= k0) hi = mid; else lo = mid + 1;
      }
      const int per = (Mc + kThreads - 1) / kThreads;
      const int j0 = min(Mc, tid * per), j1 = min(Mc, j0 + per);
      int cnt = 0;
      for (int j = j0; j < j1; ++j) cnt += key(j) <= lo;
      int tot = 0;
      int pos = block_excl_scan(cnt, sh.scan, &tot);
      for (int j = j0; j < j1; ++j)
        if (key(j) <= lo) i0l[pos++] = j;
      __syncthreads();
    }

    // -- leave-one-out predictions of the I0 members, 64 at a time
    double num = 0.0, den = 0.0;
    const int ty = tid >> 4, tx = tid & 15;
    const double inv2b = 1.0 / (2.0 * beta);
    for (int c0 = 0; c0 < k0; c0 += 64) {
      const int nc = min(64, k0 - c0);
      // (a) logits -D(y_i, y_j) / (2 beta), D from whitened dot products
      for (int j0 = 0; j0 < Mc; j0 += 64) {
        double acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
        for (int k0_ = 0; k0_ < Ny; k0_ += 16) {
          for (int e = tid; e < 16 * 64; e += kThreads) {
            const int kk = e >> 6, c = e & 63;
            const int kg = k0_ + kk;
            ga[kk * 64 + c] = (c < nc && kg < Ny) ? V[(size_t)i0l[c0 + c] * NRs + kg] : 0.0;
            gb[kk * 64 + c] = (j0 + c < Mc && kg < Ny) ? V[(size_t)(j0 + c) * NRs + kg] : 0.0;
          }
          __syncthreads();
#pragma unroll 4
          for (int kk = 0; kk < 16; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) av[x] = ga[kk * 64 + ty * 4 + x];
#pragma unroll
            for (int y = 0; y < 4; ++y) bv[y] = gb[kk * 64 + tx * 4 + y];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = 0; y < 4; ++y) acc[x][y] = fma(av[x], bv[y], acc[x][y]);
          }
          __syncthreads();
        }
#pragma unroll
        for (int x = 0; x < 4; ++x) {
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            const int c = ty * 4 + x, j = j0 + tx * 4 + y;
            if (c < nc && j < Mc) {
              const int ii = i0l[c0 + c];
              const double D = vn[ii] + vn[j] - 2.0 * acc[x][y];
              dch[(size_t)c * Mc + j] = (j == ii) ? -INFINITY : -D * inv2b;
            }
          }
        }
      }
      __syncthreads();
      // (b) row softmax (the member itself excluded): a wave per row, its
      //     lanes striding the candidates (coalesced), fixed-order wave sums
      for (int c = wave; c < nc; c += kThreads / 64) {
        double* row = dch + (size_t)c * Mc;
        double m = -INFINITY;
        for (int j = lane; j < Mc; j += 64) m = fmax(m, row[j]);
        m = wave_max_d(m);
        double s = 0.0;
        for (int j = lane; j < Mc; j += 64) {
          const double e = exp(row[j] - m);
          row[j] = e;
          s += e;
        }
        s = wave_sum(s);
        if (lane == 0) hs.rowS[c] = s;
      }
      __syncthreads();
      // (c) z~_c = sum_j e_cj z_j over the dims of x (B2) and y (Ny)
      const int nd = B2 + Ny;
      for (int d0 = 0; d0 < nd; d0 += 64) {
        double acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
        for (int k0_ = 0; k0_ < Mc; k0_ += 16) {
          // consecutive lanes take consecutive candidates (coalesced reads)
          for (int e = tid; e < 16 * 64; e += kThreads) {
            const int kk = e & 15, c = e >> 4;
            const int kg = k0_ + kk;
            ca[kk * 65 + c] = (c < nc && kg < Mc) ? dch[(size_t)c * Mc + kg] : 0.0;
            const int dd = d0 + c;
            double zv = 0.0;
            if (dd < nd && kg < Mc)
              zv = dd < B2 ? (double)xt[(size_t)dd * ldm + kg] : (double)yt[(size_t)(dd - B2) * ldm + kg];
            cb[kk * 65 + c] = zv;
          }
          __syncthreads();
#pragma unroll 4
          for (int kk = 0; kk < 16; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) av[x] = ca[kk * 65 + ty * 4 + x];
#pragma unroll
            for (int y = 0; y < 4; ++y) bv[y] = cb[kk * 65 + tx * 4 + y];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = 0; y < 4; ++y) acc[x][y] = fma(av[x], bv[y], acc[x][y]);
          }
          __syncthreads();
        }
#pragma unroll
        for (int x = 0; x < 4; ++x) {
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            const int c = ty * 4 + x, dd = d0 + tx * 4 + y;
            if (c < nc && dd < nd) {
              const int ii = i0l[c0 + c];
              const double own = dd < B2 ? (double)xt[(size_t)dd * ldm + ii]
                                         : (double)yt[(size_t)(dd - B2) * ldm + ii];
              // residual of the leave-one-out prediction: x_i - x~_i, y_i - y~_i
              zch[(size_t)c * ldz + dd] = own - acc[x][y] / hs.rowS[c];
            }
          }
        }
      }
      __syncthreads();
      // (d) c_i = A r_i; accumulate <c_i, x_i - x~_i> and ||c_i||^2
      for (int e = tid; e < nc * B2; e += kThreads) {
        const int c = e / B2, q = e - c * B2;
        const double* arow = axy + (size_t)q * NRs;
        const double* rrow = zch + (size_t)c * ldz + B2;
        double cv = 0.0;
        for (int k = 0; k < Ny; ++k) cv += arow[k] * rrow[k];
        num += cv * zch[(size_t)c * ldz + q];
        den += cv * cv;
      }
      __syncthreads();
    }
    num = block_sum_d(num, hs.red);
    den = block_sum_d(den, hs.red);
    const double alpha = den > 0.0 ? num / den : 0.0;

    // -- x0_hat = x~(beta) + alpha A (y0 - y~(beta))
    eval_eps(beta, Mc, Ny, B2, ldm, dm0, dmin, ew, yt, xt, y0v, ytil, xtil, hs);
    for (int q = tid; q < B2; q += kThreads) {
      const double* arow = axy + (size_t)q * NRs;
      double corr = 0.0;
      for (int k = 0; k < Ny; ++k) corr += arow[k] * (y0v[k] - ytil[k]);
      const double xh = xtil[q] + alpha * corr;
      const int py = q / B, px = q - py * B;
      // a block holding received pixels keeps them
      if (!partial || a.val[(size_t)(y0 + py) * p.width + x0 + px] < 0)
        a.work[(size_t)(y0 + py) * p.stride + x0 + px] = (uint8_t)fmin(fmax(floor(xh + 0.5), 0.0), 255.0);
      if (a.xhat && i < a.cap) a.xhat[(size_t)i * B2 + q] = (float)xh;
    }
    if (tid == 0) {
      a.bstate[i] = round;
      if (pend) atomicSub(pend, 1);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_hql(FrameArgs a, DevParams p, unsigned char* ws,
                                                  size_t slot_bytes) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BlockShared sh;
  __shared__ HqlShared hs;
  const RoundState* st = a.st;
  if (st->remaining == 0) return;
  const int n_hql = st->n_hql;
  if ((int)blockIdx.x >= n_hql) return;
  bool first = true;
  hql_frame(a, p, ws, slot_bytes, st->round, n_hql, first, lds_raw, sh, hs, nullptr);
}

// Every frame of a batch in turn: the workgroups (one scratch slot each)
// share each frame's HQL list.
__global__ __launch_bounds__(kThreads) void k_hql_b(BatchArgs b, DevParams p, unsigned char* ws,
                                                    size_t slot_bytes) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BlockShared sh;
  __shared__ HqlShared hs;
  if (b.bs->remaining == 0) return;
  bool first = true;
  for (int f = 0; f < b.nf; ++f) {
    const RoundState* st = b.a0.st + f;
    if (st->remaining == 0) continue;
    const int n_hql = st->n_hql;
    if ((int)blockIdx.x >= n_hql) continue;
    if (!first) __syncthreads();
    hql_frame(batch_frame(b, f), p, ws, slot_bytes, st->round, n_hql, first, lds_raw, sh, hs,
              &b.bs->pending);
  }
}

hipError_t launch_hql_b(const BatchArgs& b, const DevParams& p, unsigned char* ws,
                        size_t slot_bytes, int slots, hipStream_t s) {
  hipLaunchKernelGGL(k_hql_b, dim3(slots), dim3(kThreads), hql_lds_bytes(p), s, b, p, ws,
                     slot_bytes);
  return hipGetLastError();
}

hipError_t launch_hql(const FrameArgs& a, const DevParams& p, unsigned char* ws, size_t slot_bytes,
                      int slots, hipStream_t s) {
  hipLaunchKernelGGL(k_hql, dim3(slots), dim3(kThreads), hql_lds_bytes(p), s, a, p, ws, slot_bytes);
  return hipGetLastError();
}

hipError_t set_hql_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_hql, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_hql_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace skm
