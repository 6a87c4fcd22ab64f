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
// The dense FP64 contractions (blocked Cholesky with the explicit inverse
// factor L^-1, whitening, A = C_XY C_YY^-1, the leave-one-out distances and
// sums) run on 64 x 64 output tiles of v_mfma_f64_16x16x4f64.
// Scratch: one global slot per workgroup (layout in hql_layout).
#include "skm_device.h"

namespace skm {

struct HqlLayout {
  size_t yt, xt, cyy, axy, v, v0, y0, meany, meanx, dm0, ytil, xtil, vn, dch, zch, i0;
  size_t li, tmp;   // L^-1 (NY x NY), and a staging block of max(B^2, 64) rows
  size_t rs;        // exact byte row sums of yt, xt (and ot)
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
  h.li = take(8 * NY * NY);
  h.tmp = take(8 * (B2 > 64 ? B2 : 64) * NY);
  h.rs = take(4 * (2 * NY + B2));
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

// LDS row pitch (doubles) of the MFMA operand tiles: rows k and k + 1 of a
// tile start 128 bytes apart modulo 256, so the two half-waves of a read hit
// disjoint banks
constexpr int kTp = 80;
constexpr size_t kGemmLds = (size_t)2 * 32 * kTp * 8;
// LDS row pitch (bytes) of the int8 Gram tiles: 256 bytes of k a row, the
// 16 row starts of a half-wave's reads on distinct 4-bank groups
constexpr int kGk = 256;
constexpr int kGp8 = kGk + 16;
constexpr size_t kGramLds = (size_t)2 * 64 * kGp8;

// the diagonal block of the blocked Cholesky and its inverse, pitch 65
constexpr size_t kCholLds = (size_t)2 * 64 * 65 * 8;
// the eps_y evaluations read the candidates' context bytes from LDS when
// they fit in this much (NY x ldm bytes)
constexpr size_t kEpsLds = 96 * 1024;

__host__ __device__ inline bool hql_eps_in_lds(const HqlLayout& h) {
  return (size_t)h.ny * h.ldm <= kEpsLds;
}

// the estimation kernel's layout, with the window region large enough for
// the HQL tiles that reuse it
size_t hql_lds_bytes(const DevParams& p) {
  size_t offs[10];
  main_lds_layout(p, offs);
  const HqlLayout h = hql_layout(p);
  size_t need = (size_t)4 * p.Wd * p.Wp;
  need = need > kGemmLds ? need : kGemmLds;
  need = need > kCholLds ? need : kCholLds;
  need = need > kGramLds ? need : kGramLds;
  if (hql_eps_in_lds(h)) {
    const size_t ye = (size_t)h.ny * h.ldm;
    need = need > ye ? need : ye;
  }
  return align_up(offs[9] + need, 16);
}

// PSD repair of a pairwise-complete C_YY: lambda x 10, at most this often
constexpr int kPsdRepair = 6;
__device__ __constant__ const double kPow10[kPsdRepair + 1] = {1.0, 10.0, 100.0, 1e3, 1e4, 1e5,
                                                                1e6};

// contexts wider than this evaluate the 33 grid points of beta in one MFMA pass
constexpr int kGridPassNy = 64;
// contexts of at most kNarrowNy pixels (2 x 2 patches) whiten and form the
// leave-one-out products on VALU, a thread per candidate or per output: for
// them the 64 x 64 MFMA tiles are mostly padding and per-tile overhead
constexpr int kNarrowNy = 40;
constexpr int kNarrowNd = 48;     // and at most this many x and y coordinates
constexpr int kNarrowOut = (64 * kNarrowNd + kThreads - 1) / kThreads;

// eps_y values within this relative margin count as equal: where eps_y is
// flat (as beta -> 0 the weights become one-hot on the nearest candidate), the
// argmin of eq. epsy is not unique, so the smallest flat beta is taken and a
// refined beta must improve on it by more than the margin
constexpr double kEpsTieRel = 1e-12;

struct HqlShared {
  double red[kThreads / 64];
  double eg[33];                 // eps_y on the beta grid g = -8 .. 24
  double ginv[33];               // 1 / (2 beta_g) on that grid
  double pb[2][kThreads / 64][65];   // eval_eps_narrow: per-wave row partials, S at [64]
  int hist[kThreads];            // I0 radix selection: counts of one 8-bit digit
  long long pref;
  int rank;
  double S;
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

typedef double f64x4 __attribute__((ext_vector_type(4)));
// LDS-qualified views of the tile pointers, so that the tile traffic of
// functions that the compiler keeps out of line stays on ds_* instructions
typedef __attribute__((address_space(3))) double lds_f64;
// and global-qualified views of the scratch operands: flat loads would also
// count against the LDS wait counter and hold the tile reads behind them
template <class T>
static __device__ __forceinline__ __attribute__((address_space(1))) T* glb(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// k per staging step of gemm_f64
constexpr int kKc = 32;

// C = A B on FP64 MFMA, one workgroup, 64 x 64 output tiles in raster order.
// Wave w holds the 32 x 32 quarter (w / 2, w % 2) of a tile as 2 x 2
// v_mfma_f64_16x16x4f64 accumulators; k advances kKc at a time through LDS
// (tl: two kKc x kTp tiles).  The steps of all tiles form one pipeline: the
// operands of the next step, which may be the first of the next tile, are
// loaded into registers while the current one is multiplied.  Operands are
// read element-wise by fa(m, k) and fb(k, n); AK (BK) says that consecutive
// k of A (B) are adjacent in memory, which picks the staging order that
// keeps each wave's loads contiguous.  tiles(mt, nt, kb, ke) sets the k
// range of output tile (mt, nt) and returns false for a tile that is not
// wanted (triangular operands skip their zero blocks this way).
// epi(m, n, v) gets every output of a wanted tile once, always from the
// same lane, in a fixed order.  A tile's loads never read what an earlier
// tile's epi wrote unless the two touch disjoint rows (in-place panels).
template <bool AK, bool BK, class FA, class FB, class FT, class FE>
static __device__ void gemm_f64(int M, int N, FA fa, FB fb, FT tiles, FE epi, double* tl) {
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  lds_f64* As = (lds_f64*)tl;
  lds_f64* Bs = As + kKc * kTp;
  const int ntn = (N + 63) >> 6, nt_all = ((M + 63) >> 6) * ntn;
  const int mw = 32 * (wave >> 1), nw = 32 * (wave & 1);
  const int li = lane & 15, lk = lane >> 4;
  // staging: element s (of 8) of A is (am + (AK ? 8 s : 0), ak + (AK ? 0 : 4 s))
  const int am = AK ? (tid >> 5) : (tid & 63), ak = AK ? (tid & 31) : (tid >> 6);
  const int bn = BK ? (tid >> 5) : (tid & 63), bk = BK ? (tid & 31) : (tid >> 6);
  auto next_tile = [&](int t, int& kb, int& ke) {
    for (; t < nt_all; ++t) {
      const int mt = t / ntn, nt = t - mt * ntn;
      if (tiles(mt, nt, kb, ke)) return t;
    }
    return nt_all;
  };
  double ra[8], rb[8];
  auto load = [&](int t, int k0, int ke) {
    const int mt = t / ntn, nt = t - mt * ntn;
    const int m0 = mt * 64, n0 = nt * 64;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int m = m0 + am + (AK ? 8 * s : 0), k = k0 + ak + (AK ? 0 : 4 * s);
      ra[s] = (m < M && k < ke) ? fa(m, k) : 0.0;
      const int n = n0 + bn + (BK ? 8 * s : 0), kk = k0 + bk + (BK ? 0 : 4 * s);
      rb[s] = (n < N && kk < ke) ? fb(kk, n) : 0.0;
    }
  };
  int kb = 0, ke = 0;
  int t = next_tile(0, kb, ke);
  if (t < nt_all) {
    int k0 = kb;
    load(t, k0, ke);
    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
    while (true) {
      __syncthreads();                       // the previous step's reads are done
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        As[(ak + (AK ? 0 : 4 * s)) * kTp + am + (AK ? 8 * s : 0)] = ra[s];
        Bs[(bk + (BK ? 0 : 4 * s)) * kTp + bn + (BK ? 8 * s : 0)] = rb[s];
      }
      __syncthreads();
      // the next step: the tile's next k range, else the next wanted tile
      int t2 = t, k2 = k0 + kKc, kb2 = kb, ke2 = ke;
      const bool last = k2 >= ke;
      if (last) {
        t2 = next_tile(t + 1, kb2, ke2);
        k2 = kb2;
      }
      if (t2 < nt_all) load(t2, k2, ke2);
#pragma unroll
      for (int k4 = 0; k4 < kKc / 4; ++k4) {
        const lds_f64* ar = As + (4 * k4 + lk) * kTp;
        const lds_f64* br = Bs + (4 * k4 + lk) * kTp;
        const double a0 = ar[mw + li], a1 = ar[mw + 16 + li];
        const double b0 = br[nw + li], b1 = br[nw + 16 + li];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
      if (last) {
        // accumulator layout of v_mfma_f64_16x16x4f64: lane l, element r
        // holds row l / 16 + 4 r, column l % 16 of its 16 x 16 block
        const int mt = t / ntn, nt = t - mt * ntn;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int m = mt * 64 + mw + 16 * x + lk + 4 * r, n = nt * 64 + nw + 16 * y + li;
              if (m < M && n < N) epi(m, n, acc[x][y][r]);
            }
            acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
          }
        if (t2 >= nt_all) break;
      }
      t = t2; k0 = k2; kb = kb2; ke = ke2;
    }
  }
  __syncthreads();
}

// C (n x n, row stride ld, lower triangle) = L L^T by 64-wide block columns,
// right-looking: the diagonal block is factored in LDS and inverted there;
// the panel below it, L_ik = C_ik L_kk^-T, and the trailing update
// C_ij -= L_ik L_jk^T run on gemm_f64.  Then Li = L^-1 (lower, zeros above
// the diagonal inside the diagonal blocks) block row by block row:
// Li_ik = -L_ii^-1 sum_{k <= m < i} L_im Li_mk.  C's strictly lower blocks
// end up holding L.  Returns false, uniformly, at the first pivot that is
// not positive.  tmp: 64 x ld doubles; lds: kCholLds bytes.
static __device__ bool chol_inv(double* C, int ld, int n, double* Li, double* tmp, double* lds) {
  const int tid = threadIdx.x;
  lds_f64* D = (lds_f64*)lds;
  lds_f64* Di = D + 64 * 65;
  const int nb = (n + 63) >> 6;
  for (int kb = 0; kb < nb; ++kb) {
    const int k0 = 64 * kb, kn = min(64, n - k0);
    for (int e = tid; e < 64 * 64; e += kThreads) {
      const int i = e >> 6, j = e & 63;
      D[i * 65 + j] = (i < kn && j <= i) ? C[(size_t)(k0 + i) * ld + k0 + j] : 0.0;
      Di[i * 65 + j] = 0.0;
    }
    __syncthreads();
    // unblocked right-looking factorisation of the diagonal block; column j
    // is scaled after the barrier that ends its trailing update (nobody
    // reads it then)
    for (int j = 0; j < kn; ++j) {
      const double dd = D[j * 65 + j];
      if (!(dd > 0.0)) return false;          // uniform: written before a barrier
      const double d = sqrt(dd), inv = 1.0 / d;
      for (int e = tid; e < 64 * 64; e += kThreads) {
        const int i = e >> 6, l = e & 63;
        if (l > j && l <= i && i < kn)
          D[i * 65 + l] -= (D[i * 65 + j] * inv) * (D[l * 65 + j] * inv);
      }
      __syncthreads();
      for (int i = j + tid; i < kn; i += kThreads) D[i * 65 + j] = i == j ? d : D[i * 65 + j] * inv;
    }
    __syncthreads();
    // Di = D^-1 row by row: Di_ic = (delta_ic - sum_{c <= m < i} D_im Di_mc) / D_ii,
    // four lanes per column c, each over every fourth m
    {
      const int c = tid >> 2, part = tid & 3;
      for (int i = 0; i < kn; ++i) {
        double s = 0.0;
        if (c < i)
          for (int m = c + part; m < i; m += 4) s += D[i * 65 + m] * Di[m * 65 + c];
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        if (part == 0 && c <= i) Di[i * 65 + c] = ((i == c ? 1.0 : 0.0) - s) / D[i * 65 + i];
        __syncthreads();
      }
    }
    for (int e = tid; e < kn * 64; e += kThreads) {
      const int i = e >> 6, c = e & 63;
      if (c < kn) Li[(size_t)(k0 + i) * ld + k0 + c] = Di[i * 65 + c];
    }
    __syncthreads();
    const int r0 = k0 + 64, nr = n - r0;
    if (nr <= 0) continue;
    // panel: L_ik[i][c] = sum_m C_ik[i][m] Di[c][m]  (in place, row tiles disjoint)
    gemm_f64<true, true>(
        nr, kn, [=](int i, int m) { return glb(C)[(size_t)(r0 + i) * ld + k0 + m]; },
        [=](int m, int c) { return glb(Li)[(size_t)(k0 + c) * ld + k0 + m]; },
        [=](int, int, int& kb_, int& ke_) { kb_ = 0; ke_ = kn; return true; },
        [=](int i, int c, double v) { glb(C)[(size_t)(r0 + i) * ld + k0 + c] = v; }, lds);
    // trailing update of the lower tiles
    gemm_f64<true, true>(
        nr, nr, [=](int i, int m) { return glb(C)[(size_t)(r0 + i) * ld + k0 + m]; },
        [=](int m, int l) { return glb(C)[(size_t)(r0 + l) * ld + k0 + m]; },
        [=](int mt, int nt, int& kb_, int& ke_) { kb_ = 0; ke_ = kn; return nt <= mt; },
        [=](int i, int l, double v) { glb(C)[(size_t)(r0 + i) * ld + r0 + l] -= v; }, lds);
  }
  for (int ib = 1; ib < nb; ++ib) {
    const int i0 = 64 * ib, in = min(64, n - i0);
    // S = L[i0 .., 0 .. i0) Li[0 .. i0, 0 .. i0), then Li[i0 .., 0 .. i0) = -Di S
    gemm_f64<true, false>(
        in, i0, [=](int r, int m) { return glb(C)[(size_t)(i0 + r) * ld + m]; },
        [=](int m, int c) { return glb(Li)[(size_t)m * ld + c]; },
        [=](int, int nt, int& kb_, int& ke_) { kb_ = 64 * nt; ke_ = i0; return true; },
        [=](int r, int c, double v) { glb(tmp)[(size_t)r * ld + c] = v; }, lds);
    gemm_f64<true, false>(
        in, i0, [=](int r, int m) { return glb(Li)[(size_t)(i0 + r) * ld + i0 + m]; },
        [=](int m, int c) { return glb(tmp)[(size_t)m * ld + c]; },
        [=](int, int, int& kb_, int& ke_) { kb_ = 0; ke_ = in; return true; },
        [=](int r, int c, double v) { glb(Li)[(size_t)(i0 + r) * ld + c] = -v; }, lds);
  }
  return true;
}

// Sums of eight per-lane values over a wave in ten lane exchanges: after
// halving steps over lane bits 5, 4, 3 each lane carries one of the eight
// rows, then bits 2..0 finish the sum.  Lane 8 c returns row c's total
// (c = bits 5..3 of the lane).  The order is fixed.
static __device__ __forceinline__ double reduce8(const double (&v)[8]) {
  const int lane = lane_id();
  const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0, h3 = (lane & 8) != 0;
  double u[4], w[2];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    u[r] = (h5 ? v[r + 4] : v[r]) + __shfl_xor(h5 ? v[r] : v[r + 4], 32, 64);
#pragma unroll
  for (int r = 0; r < 2; ++r)
    w[r] = (h4 ? u[r + 2] : u[r]) + __shfl_xor(h4 ? u[r] : u[r + 2], 16, 64);
  double x = (h3 ? w[1] : w[0]) + __shfl_xor(h3 ? w[0] : w[1], 8, 64);
  x += __shfl_xor(x, 4, 64);
  x += __shfl_xor(x, 2, 64);
  x += __shfl_xor(x, 1, 64);
  return x;
}

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Exact row sums of a byte matrix (R rows of ld bytes, ld a multiple of 16,
// rows 16-byte aligned): a wave per row.
static __device__ void byte_row_sums(const uint8_t* P, int R, int ld, int* out) {
  const int lane = lane_id(), wave = wave_id();
  for (int a = wave; a < R; a += kThreads / 64) {
    const uint4* row = reinterpret_cast<const uint4*>(P + (size_t)a * ld);
    uint32_t s = 0;
    for (int c = lane; c < ld / 16; c += 64) {
      const uint4 v = row[c];
      s = __builtin_amdgcn_udot4(v.x, 0x01010101u, s, false);
      s = __builtin_amdgcn_udot4(v.y, 0x01010101u, s, false);
      s = __builtin_amdgcn_udot4(v.z, 0x01010101u, s, false);
      s = __builtin_amdgcn_udot4(v.w, 0x01010101u, s, false);
    }
    const int t = wave_sum((int)s);
    if (lane == 0) out[a] = t;
  }
}

// Exact integer Gram G = P Q^T of two u8 row sets (R1 and R2 rows of ld
// bytes, zero padded, ld a multiple of 64) on v_mfma_i32_16x16x64_i8.  The
// bytes enter the signed product as p - 128, so that
//   sum_k p_k q_k = sum_k (p_k - 128)(q_k - 128) + 128 (sp + sq) - 128^2 ld
// with the exact row sums sp[i], sq[j]; every term stays below 2^31 for
// ld <= 2^16.  64 x 64 output tiles (with sym, P == Q and only tiles on or
// below the diagonal), k staged kGk bytes at a time through LDS (t8:
// kGramLds bytes); wave w holds the 32 x 32 quarter (w / 2, w % 2) as 2 x 2
// accumulators whose element r of lane l is row 4 (l / 16) + r, column
// l % 16.  epi(i, j, g) gets each entry of a computed tile once.
template <class FE>
static __device__ void gram_i8(const uint8_t* P, const uint8_t* Q, int R1, int R2, int ld,
                               const int* sp, const int* sq, bool sym, FE epi, uint8_t* t8) {
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  uint8_t* ta = t8;
  uint8_t* tb = t8 + 64 * kGp8;
  const int nt1 = (R1 + 63) / 64, nt2 = (R2 + 63) / 64;
  const int mw = 32 * (wave >> 1), nw = 32 * (wave & 1);
  const int li = lane & 15, lk = lane >> 4;
  const int srow = tid >> 2, sseg = tid & 3;      // staging: 4 x 16 bytes per thread and operand
  const int corr = 16384 * ld;
  for (int t1 = 0; t1 < nt1; ++t1) {
    for (int t2 = 0; t2 < nt2; ++t2) {
      if (sym && t2 > t1) continue;
      i32x4 acc[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = i32x4{0, 0, 0, 0};
      const int r1 = t1 * 64 + srow, r2 = t2 * 64 + srow;
      for (int kk = 0; kk < ld; kk += kGk) {
        uint4 va[4], vb[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = kk + 16 * (sseg + 4 * s);
          uint4 a = {0u, 0u, 0u, 0u}, b = {0u, 0u, 0u, 0u};
          if (k < ld) {
            if (r1 < R1) a = *reinterpret_cast<const uint4*>(P + (size_t)r1 * ld + k);
            if (r2 < R2) b = *reinterpret_cast<const uint4*>(Q + (size_t)r2 * ld + k);
            a.x ^= 0x80808080u; a.y ^= 0x80808080u; a.z ^= 0x80808080u; a.w ^= 0x80808080u;
            b.x ^= 0x80808080u; b.y ^= 0x80808080u; b.z ^= 0x80808080u; b.w ^= 0x80808080u;
          }
          va[s] = a;
          vb[s] = b;
        }
        __syncthreads();                       // the previous step's reads are done
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          *reinterpret_cast<uint4*>(ta + srow * kGp8 + 16 * (sseg + 4 * s)) = va[s];
          *reinterpret_cast<uint4*>(tb + srow * kGp8 + 16 * (sseg + 4 * s)) = vb[s];
        }
        __syncthreads();
#pragma unroll
        for (int k64 = 0; k64 < kGk / 64; ++k64) {
          const int ko = 64 * k64 + 16 * lk;
          const i32x4 a0 = *reinterpret_cast<const i32x4*>(ta + (mw + li) * kGp8 + ko);
          const i32x4 a1 = *reinterpret_cast<const i32x4*>(ta + (mw + 16 + li) * kGp8 + ko);
          const i32x4 b0 = *reinterpret_cast<const i32x4*>(tb + (nw + li) * kGp8 + ko);
          const i32x4 b1 = *reinterpret_cast<const i32x4*>(tb + (nw + 16 + li) * kGp8 + ko);
          acc[0][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b1, acc[1][1], 0, 0, 0);
        }
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = t1 * 64 + mw + 16 * x + 4 * lk + r, j = t2 * 64 + nw + 16 * y + li;
            if (i < R1 && j < R2) epi(i, j, acc[x][y][r] + 128 * (sp[i] + sq[j]) - corr);
          }
    }
  }
  __syncthreads();
}

// One evaluation of eps_y(beta) (eq. epsy): weights e_j = exp(-dm0_j/(2 beta)
// - max), S = sum e_j, y~ = sum e_j y_j / S; returns ||y0 - y~||^2.  Leaves
// ew, S (in hs.S) and ytil for the caller.  With xt != nullptr also x~.
// ys: the candidates' context bytes (Ny rows of ldm, zero padded; in LDS
// with YL, else in global memory, where xt is too).  A wave takes eight rows at a time; a lane takes four
// consecutive candidates of four 256-candidate strips per step (32 loads in
// flight), then reduce8 sums the rows.
typedef __attribute__((address_space(3))) const uint32_t lds_u32c;
typedef __attribute__((address_space(1))) const uint32_t glb_u32c;

template <bool YL>
static __device__ double eval_eps(double beta, int Mc, int Ny, int B2, int ldm, const double* dm0,
                                  double dmin, double* ew_, const uint8_t* ys, const uint8_t* xt,
                                  const double* y0, double* ytil, double* xtil, HqlShared& hs) {
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  lds_f64* ew = (lds_f64*)ew_;
  const double inv2b = 1.0 / (2.0 * beta);      // one division per evaluation
  const double m = -dmin * inv2b;
  double s = 0.0;
  for (int j = tid; j < Mc; j += kThreads) {
    const double e = exp(-glb(dm0)[j] * inv2b - m);
    ew[j] = e;
    s += e;
  }
  const double S = block_sum_d(s, hs.red);     // barrier: ew visible
  const int R = xt ? Ny + B2 : Ny;
  double part = 0.0;
  for (int a0 = 8 * wave; a0 < R; a0 += 8 * (kThreads / 64)) {
    const uint8_t* rp[8];
    bool ok[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int a = a0 + r;
      ok[r] = a < R;
      rp[r] = a < Ny ? ys + (size_t)a * ldm : xt + (size_t)(a < R ? a - Ny : 0) * ldm;
    }
    double acc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = 0.0;
    for (int j0 = 4 * lane; j0 < Mc; j0 += 1024) {
      uint32_t w[4][8];
      double e[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + 256 * q;
#pragma unroll
        for (int t = 0; t < 4; ++t) e[q][t] = j + t < Mc ? ew[j + t] : 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r)
          w[q][r] = (ok[r] && j < Mc) ? (YL ? *(lds_u32c*)(rp[r] + j) : *(glb_u32c*)(rp[r] + j)) : 0u;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 8; ++r)
          acc[r] += e[q][0] * (double)(w[q][r] & 0xffu) + e[q][1] * (double)((w[q][r] >> 8) & 0xffu) +
                    e[q][2] * (double)((w[q][r] >> 16) & 0xffu) + e[q][3] * (double)(w[q][r] >> 24);
    }
    const double tot = reduce8(acc);
    if ((lane & 7) == 0) {
      const int a = a0 + (lane >> 3);
      if (a < Ny) {
        const double yv = tot / S;
        glb(ytil)[a] = yv;
        const double d = glb(y0)[a] - yv;
        part += d * d;
      } else if (a < R) {
        glb(xtil)[a - Ny] = tot / S;
      }
    }
  }
  hs.S = S;
  return block_sum_d(part, hs.red);
}

// eps_y(beta) for contexts of at most 64 pixels (2 x 2 patches): wave w
// takes the w-th quarter of the candidates for every context row, keeping its
// weights in registers, and leaves per-row partial sums and its share of S in
// hs.pb[flip][w]; after one barrier every wave adds the four partials in
// wave order and returns the same eps_y.  Alternating between the two
// halves of pb (flip) keeps a wave from overwriting partials that another
// wave has yet to read.  Same weights and sums as eval_eps, in another
// order; y~ is not kept.
template <bool YL>
static __device__ double eval_eps_narrow(double beta, int Mc, int Ny, int ldm, const double* dm0,
                                         double dmin, const uint8_t* ys, const double* y0,
                                         HqlShared& hs, int flip) {
  const int lane = lane_id(), wave = wave_id();
  const double inv2b = 1.0 / (2.0 * beta);
  const double m = -dmin * inv2b;
  const int Q = ((Mc + 4 * 64 - 1) / (4 * 64)) * 64;        // candidates per wave, multiple of 64
  const int c0 = wave * Q, c1 = min(Mc, c0 + Q);
  constexpr int kSteps = (kMaxPer * kThreads + 4 * 256 - 1) / (4 * 256);
  double e[kSteps][4];
  double sp = 0.0;
#pragma unroll
  for (int st = 0; st < kSteps; ++st) {
    const int j0 = c0 + 4 * lane + 256 * st;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = j0 + t;
      e[st][t] = j < c1 ? exp(-glb(dm0)[j] * inv2b - m) : 0.0;
      sp += e[st][t];
    }
  }
  sp = wave_sum(sp);
  lds_f64* pb = (lds_f64*)&hs.pb[flip][wave][0];
  for (int a0 = 0; a0 < Ny; a0 += 8) {
    double acc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = 0.0;
#pragma unroll
    for (int st = 0; st < kSteps; ++st) {
      const int j0 = c0 + 4 * lane + 256 * st;
      if (c0 + 256 * st < c1) {                    // wave-uniform
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const uint8_t* row = ys + (size_t)(a0 + r) * ldm + j0;
          const uint32_t w = (a0 + r < Ny && j0 < c1)
                                 ? (YL ? *(lds_u32c*)row : *(glb_u32c*)row) : 0u;
          acc[r] += e[st][0] * (double)(w & 0xffu) + e[st][1] * (double)((w >> 8) & 0xffu) +
                    e[st][2] * (double)((w >> 16) & 0xffu) + e[st][3] * (double)(w >> 24);
        }
      }
    }
    const double tot = reduce8(acc);
    const int a = a0 + (lane >> 3);
    if ((lane & 7) == 0 && a < Ny) pb[a] = tot;
  }
  if (lane == 0) pb[64] = sp;
  __syncthreads();
  const lds_f64* q0 = (const lds_f64*)&hs.pb[flip][0][0];
  const lds_f64* q1 = q0 + 65;
  const lds_f64* q2 = q1 + 65;
  const lds_f64* q3 = q2 + 65;
  const double S = ((q0[64] + q1[64]) + q2[64]) + q3[64];
  double part = 0.0;
  if (lane < Ny) {
    const double d = glb(y0)[lane] - (((q0[lane] + q1[lane]) + q2[lane]) + q3[lane]) / S;
    part = d * d;
  }
  return wave_sum(part);
}

// The 33 grid evaluations of eps_y for contexts of at most 32 pixels: a wave
// per beta_g over all candidates, with no barrier inside (the weights and
// sums of eval_eps_narrow, one wave instead of four); eps_g to hs.eg[g].
// 1 / (2 beta_g) comes from hs.ginv.
template <bool YL>
static __device__ void grid_eps_narrow(int Mc, int Ny, int ldm, const double* dm0, double dmin,
                                       const uint8_t* ys, const double* y0, HqlShared& hs) {
  const int lane = lane_id(), wave = wave_id();
  for (int g = wave; g < 33; g += kThreads / 64) {
    const double inv2b = hs.ginv[g];
    const double m = -dmin * inv2b;
    double acc[32];
#pragma unroll
    for (int a = 0; a < 32; ++a) acc[a] = 0.0;
    double sp = 0.0;
    for (int j0 = 4 * lane; j0 < Mc; j0 += 256) {
      double e[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        e[t] = j0 + t < Mc ? exp(-glb(dm0)[j0 + t] * inv2b - m) : 0.0;
        sp += e[t];
      }
#pragma unroll
      for (int a = 0; a < 32; ++a) {
        const uint8_t* row = ys + (size_t)a * ldm + j0;
        const uint32_t w = a < Ny ? (YL ? *(lds_u32c*)row : *(glb_u32c*)row) : 0u;
        acc[a] += e[0] * (double)(w & 0xffu) + e[1] * (double)((w >> 8) & 0xffu) +
                  e[2] * (double)((w >> 16) & 0xffu) + e[3] * (double)(w >> 24);
      }
    }
    // butterfly: lane l ends with the wave's sum of row l >> 1
    double u[16], v[8], x[4], q[2];
    const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0, h3 = (lane & 8) != 0,
               h2 = (lane & 4) != 0, h1 = (lane & 2) != 0;
#pragma unroll
    for (int r = 0; r < 16; ++r)
      u[r] = (h5 ? acc[r + 16] : acc[r]) + __shfl_xor(h5 ? acc[r] : acc[r + 16], 32, 64);
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = (h4 ? u[r + 8] : u[r]) + __shfl_xor(h4 ? u[r] : u[r + 8], 16, 64);
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = (h3 ? v[r + 4] : v[r]) + __shfl_xor(h3 ? v[r] : v[r + 4], 8, 64);
#pragma unroll
    for (int r = 0; r < 2; ++r) q[r] = (h2 ? x[r + 2] : x[r]) + __shfl_xor(h2 ? x[r] : x[r + 2], 4, 64);
    double t = (h1 ? q[1] : q[0]) + __shfl_xor(h1 ? q[0] : q[1], 2, 64);
    t += __shfl_xor(t, 1, 64);
    const double S = wave_sum(sp);
    const int a = lane >> 1;
    double part = 0.0;
    if ((lane & 1) == 0 && a < Ny) {
      const double d = glb(y0)[a] - t / S;
      part = d * d;
    }
    part = wave_sum(part);
    if (lane == 0) hs.eg[g] = part;
  }
}

// Narrow-context whitening (Ny <= NYN): a thread per candidate with its NYN
// context values in registers; L^-1 (NYN x NYN, zeros above the diagonal and
// beyond Ny) in LDS, read by every lane at once.  Writes V[j], dm0[j], vn[j]
// and v0; returns the thread's smallest distance to y0.
template <int NYN>
static __device__ __forceinline__ double whiten_narrow(const double* Li, int NRs, int Ny,
                                                       const uint8_t* yt, int ldm, int Mc,
                                                       const double* y0v, double* V, double* v0,
                                                       double* dm0, double* vn, double* tl) {
  const int tid = threadIdx.x;
  lds_f64* lw = (lds_f64*)tl;
  lds_f64* lv0 = lw + NYN * NYN;
  for (int e = tid; e < NYN * NYN; e += kThreads) {
    const int aa = e / NYN, k = e - aa * NYN;
    lw[e] = (aa < Ny && k <= aa) ? glb(Li)[(size_t)aa * NRs + k] : 0.0;
  }
  __syncthreads();
  if (tid < Ny) {
    double v = 0.0;
    for (int k = 0; k <= tid; ++k) v = fma(lw[tid * NYN + k], glb(y0v)[k], v);
    lv0[tid] = v;
    glb(v0)[tid] = v;
  }
  __syncthreads();
  double dmin = INFINITY;
  for (int j = tid; j < Mc; j += kThreads) {
    double y[NYN];
#pragma unroll
    for (int k = 0; k < NYN; ++k) y[k] = k < Ny ? (double)glb(yt)[(size_t)k * ldm + j] : 0.0;
    double sd = 0.0, nn = 0.0;
    for (int aa = 0; aa < Ny; ++aa) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < NYN; ++k) v = fma(lw[aa * NYN + k], y[k], v);
      glb(V)[(size_t)j * NRs + aa] = v;
      const double d = v - lv0[aa];
      sd += d * d;
      nn += v * v;
    }
    glb(dm0)[j] = sd;
    glb(vn)[j] = nn;
    dmin = fmin(dmin, sd);
  }
  return dmin;
}

// Narrow-context leave-one-out logits -D(y_i, y_j) / (2 beta) for the nc
// members from c0 on: a thread per candidate with its whitened row in
// registers; the members' rows, norms and indices in LDS.
template <int NYN>
static __device__ __forceinline__ void logits_narrow(const double* V, const int* i0l, int c0,
                                                     int nc, int NRs, int Ny, const double* vn,
                                                     int Mc, double* dch, double inv2b,
                                                     double* tl) {
  const int tid = threadIdx.x;
  lds_f64* vi = (lds_f64*)tl;                          // nc x NYN
  lds_f64* vni = vi + 64 * NYN;                       // their squared norms
  __attribute__((address_space(3))) int* iic = (__attribute__((address_space(3))) int*)(vni + 64);
  for (int e = tid; e < nc * NYN; e += kThreads) {
    const int c = e / NYN, k = e - c * NYN;
    vi[e] = k < Ny ? glb(V)[(size_t)glb(i0l)[c0 + c] * NRs + k] : 0.0;
  }
  if (tid < nc) {
    const int ii = glb(i0l)[c0 + tid];
    iic[tid] = ii;
    vni[tid] = glb(vn)[ii];
  }
  __syncthreads();
  for (int j = tid; j < Mc; j += kThreads) {
    double vj[NYN];
#pragma unroll
    for (int k = 0; k < NYN; ++k) vj[k] = k < Ny ? glb(V)[(size_t)j * NRs + k] : 0.0;
    const double vnj = glb(vn)[j];
    for (int c = 0; c < nc; ++c) {
      double g = 0.0;
#pragma unroll
      for (int k = 0; k < NYN; ++k) g = fma(vi[c * NYN + k], vj[k], g);
      glb(dch)[(size_t)c * Mc + j] = (j == iic[c]) ? -INFINITY : -(vni[c] + vnj - 2.0 * g) * inv2b;
    }
  }
  __syncthreads();
}

// HQL for entry h of one frame's list, on this workgroup's scratch slot.
// The caller has run phase_tables; `first` is true for the workgroup's first
// block of the launch.
static __device__ __forceinline__ void hql_block(const FrameArgs& a, const DevParams& p,
                                                 unsigned char* ws, size_t slot_bytes, int round,
                                                 int h, bool first, unsigned char* lds_raw,
                                                 BlockShared& sh, HqlShared& hs, int* pend) {
  const MainLds L = carve_main_lds(lds_raw, p);
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int B = p.B, r = p.r, W = p.W, Wd = p.Wd, Wp = p.Wp;
  const int B2 = B * B;
  const int qbase = W * Wp + W;
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
  double* Li = (double*)(slot + hl.li);
  double* tmp = (double*)(slot + hl.tmp);
  int* rsy = (int*)(slot + hl.rs);
  int* rso = rsy + hl.ny;
  int* rsx = rso + hl.ny;
  const int ldm = hl.ldm, ldz = hl.ldz, NRs = hl.ny;      // NRs: row stride of Ny rows

  // LDS reuse once the window has been gathered
  uint8_t* t8 = (uint8_t*)L.winp;                    // int8 Gram tiles
  double* tl = (double*)L.winp;                      // MFMA operand tiles / Cholesky blocks
  uint16_t* m0off = (uint16_t*)L.qu;                 // known ring pixels (footprint offsets)
  uint16_t* compo = L.selo;                          // complete candidates: window offset
  int* compd = (int*)L.selw;                         //   and exact Euclidean distance

  {
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
      const int off = (r + q / B) * Wp + r + (q % B);
      for (int k = lane; k < ldm; k += 64)
        xt[(size_t)q * ldm + k] = k < Mc ? (uint8_t)(L.winp[compo[k] + off] & 0xffu) : (uint8_t)0;
    }
    for (int aa = tid; aa < Ny; aa += kThreads)
      y0v[aa] = (double)(int)(int16_t)(L.winp[qbase + m0off[aa]] & 0xffffu);
    __syncthreads();
    if (!hp) {
      // column means from exact integer row sums
      byte_row_sums(yt, Ny, ldm, rsy);
      byte_row_sums(xt, B2, ldm, rsx);
      __syncthreads();
      for (int aa = tid; aa < Ny; aa += kThreads) meany[aa] = (double)rsy[aa] / (double)Mc;
      for (int q = tid; q < B2; q += kThreads) meanx[q] = (double)rsx[q] / (double)Mc;
      __syncthreads();

      // -- covariance blocks C_YY (Ny x Ny) and C_XY (B2 x Ny), 1/M
      //    normalised: G / M - mean_i mean_j from the exact integer Grams
      const double invM = 1.0 / (double)Mc;
      gram_i8(yt, yt, Ny, Ny, ldm, rsy, rsy, true,
              [=](int i, int j, int g) {
                const double c = (double)g * invM - glb(meany)[i] * glb(meany)[j];
                glb(cyy)[(size_t)i * NRs + j] = c;
                glb(cyy)[(size_t)j * NRs + i] = c;
              }, t8);
      gram_i8(xt, yt, B2, Ny, ldm, rsx, rsy, false,
              [=](int q, int j, int g) { glb(axy)[(size_t)q * NRs + j] = (double)g * invM - glb(meanx)[q] * glb(meany)[j]; },
              t8);
    } else {
      // -- pairwise-complete covariance: for coordinates a, b the candidates
      //    knowing both (N_ab of them); exact integer Grams of the values
      //    (unknown = 0) and of the availability, then
      //    C_ab = G_ab / N_ab - S_a(b) S_b(a) / N_ab^2 with S_a(b) the sum of
      //    coordinate a over those candidates (0 where N_ab = 0).  The x
      //    coordinates are always known: N_qb = N_bb.
      byte_row_sums(yt, Ny, ldm, rsy);
      byte_row_sums(xt, B2, ldm, rsx);
      byte_row_sums(ot, Ny, ldm, rso);
      __syncthreads();
      gram_i8(yt, yt, Ny, Ny, ldm, rsy, rsy, true,
              [=](int i, int j, int g) {
                glb(cyy)[(size_t)i * NRs + j] = (double)g;
                glb(cyy)[(size_t)j * NRs + i] = (double)g;
              }, t8);
      gram_i8(ot, ot, Ny, Ny, ldm, rso, rso, true,
              [=](int i, int j, int g) { glb(gn)[i * Ny + j] = g; glb(gn)[j * Ny + i] = g; }, t8);
      gram_i8(yt, ot, Ny, Ny, ldm, rsy, rso, false,
              [=](int i, int j, int g) { glb(gs)[i * Ny + j] = g; }, t8);
      gram_i8(xt, yt, B2, Ny, ldm, rsx, rsy, false,
              [=](int q, int j, int g) { glb(axy)[(size_t)q * NRs + j] = (double)g; }, t8);
      gram_i8(xt, ot, B2, Ny, ldm, rsx, rso, false,
              [=](int q, int j, int g) { glb(gsx)[q * Ny + j] = g; }, t8);
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

    // -- ridge, then C_YY + lambda I = L L^T and Li = L^-1 (chol_inv).
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
    bool factored = false;
    for (int rep = 0; rep <= (hp ? kPsdRepair : 0); ++rep) {
      if (rep > 0) {
        for (int e = tid; e < Ny * Ny; e += kThreads) {
          const int aa = e / Ny, bb = e - aa * Ny;
          cyy[(size_t)aa * NRs + bb] = cyy0[e];
        }
        __syncthreads();
      }
      const double lam = lam0 * kPow10[rep];
      for (int aa = tid; aa < Ny; aa += kThreads) cyy[(size_t)aa * NRs + aa] += lam;
      __syncthreads();
      factored = chol_inv(cyy, NRs, Ny, Li, tmp, tl);
      __syncthreads();
      if (factored) break;
    }
    if (!factored) {
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
      return;
    }

    // -- A = C_XY C_YY^-1 = (C_XY L^-T) L^-1: T in tmp, then A over C_XY
    gemm_f64<true, true>(
        B2, Ny, [=](int q, int k) { return glb(axy)[(size_t)q * NRs + k]; },
        [=](int k, int ii) { return glb(Li)[(size_t)ii * NRs + k]; },
        [=](int, int nt, int& kb_, int& ke_) { kb_ = 0; ke_ = min(Ny, 64 * nt + 64); return true; },
        [=](int q, int ii, double v) { glb(tmp)[(size_t)q * NRs + ii] = v; }, tl);
    gemm_f64<true, false>(
        B2, Ny, [=](int q, int ii) { return glb(tmp)[(size_t)q * NRs + ii]; },
        [=](int ii, int mm) { return glb(Li)[(size_t)ii * NRs + mm]; },
        [=](int, int nt, int& kb_, int& ke_) { kb_ = 64 * nt; ke_ = Ny; return true; },
        [=](int q, int mm, double v) { glb(axy)[(size_t)q * NRs + mm] = v; }, tl);
    // -- whitening: V[j] = L^-1 y_j for every candidate (row j of V), v0 =
    //    L^-1 y0, and the Mahalanobis distances to y0 and squared norms of the
    //    whitened candidates
    double dmin = INFINITY;
    if (Ny <= kNarrowNy) {
      // a thread per candidate, L^-1 in LDS (every lane reads the same entry)
      dmin = Ny <= 32 ? whiten_narrow<32>(Li, NRs, Ny, yt, ldm, Mc, y0v, V, v0, dm0, vn, tl)
                      : whiten_narrow<kNarrowNy>(Li, NRs, Ny, yt, ldm, Mc, y0v, V, v0, dm0, vn, tl);
    } else {
      // column tile nt of V needs k < 64 (nt + 1)
      gemm_f64<false, true>(
          Mc + 1, Ny,
          [=](int j, int k) { return j < Mc ? (double)glb(yt)[(size_t)k * ldm + j] : glb(y0v)[k]; },
          [=](int k, int aa) { return glb(Li)[(size_t)aa * NRs + k]; },
          [=](int, int nt, int& kb_, int& ke_) { kb_ = 0; ke_ = min(Ny, 64 * nt + 64); return true; },
          [=](int j, int aa, double v) { (j < Mc ? glb(V) + (size_t)j * NRs : glb(v0))[aa] = v; }, tl);
      for (int j = tid; j < Mc; j += kThreads) {
        const double* row = V + (size_t)j * NRs;
        double sd = 0.0, nn = 0.0;
        for (int k = 0; k < Ny; ++k) {
          const double d = row[k] - v0[k];
          sd += d * d;
          nn += row[k] * row[k];
        }
        dm0[j] = sd;
        vn[j] = nn;
        dmin = fmin(dmin, sd);
      }
    }
    dmin = block_min_d(dmin, hs.red);

    // -- beta grid D0 2^(g/2), g = -8 .. 24.  With wide contexts the 33
    //    evaluations of eps_y run in one pass: E[g][j] = exp(-dm0_j / (2 beta_g)
    //    - max) (the weights of eval_eps) into the leave-one-out logit rows,
    //    then [T | S] = E [Y^T | 1] on the MFMA tiles, and
    //    eps_g = ||y0 - T_g / S_g||^2, a wave per g.  Contexts of at most 32
    //    pixels (2 x 2 patches) take a wave per g over all candidates
    //    (grid_eps_narrow, after the LDS copy below), the others up to 64
    //    pixels 33 eval_eps calls.
    const double D0 = fmax(dmin, 1e-9);
    if (Ny > kGridPassNy) {
      if (tid < 33) hs.ginv[tid] = 1.0 / (2.0 * (D0 * exp2((double)(tid - 8) / 2.0)));
      __syncthreads();
      for (int g = 0; g < 33; ++g) {
        const double inv2b = hs.ginv[g];
        const double m = -dmin * inv2b;
        for (int j = tid; j < Mc; j += kThreads)
          glb(dch)[(size_t)g * Mc + j] = exp(-glb(dm0)[j] * inv2b - m);
      }
      __syncthreads();
      gemm_f64<true, true>(
          33, Ny + 1, [=](int g, int j) { return glb(dch)[(size_t)g * Mc + j]; },
          [=](int j, int aa) { return aa < Ny ? (double)glb(yt)[(size_t)aa * ldm + j] : 1.0; },
          [=](int, int, int& kb_, int& ke_) { kb_ = 0; ke_ = Mc; return true; },
          [=](int g, int aa, double v) { glb(tmp)[(size_t)g * NRs + aa] = v; }, tl);
      for (int g = wave; g < 33; g += kThreads / 64) {
        const double* row = tmp + (size_t)g * NRs;
        const double S = row[Ny];
        double part = 0.0;
        for (int aa = lane; aa < Ny; aa += 64) {
          const double d = y0v[aa] - row[aa] / S;
          part += d * d;
        }
        part = wave_sum(part);
        if (lane == 0) hs.eg[g] = part;
      }
      __syncthreads();
    }
    // -- the candidates' context bytes for the eps_y evaluations: an LDS
    //    copy when they fit (the operand tiles are idle until the
    //    leave-one-out sums)
    const bool yl = hql_eps_in_lds(hl);
    if (yl) {
      uint4* dst = (uint4*)L.winp;
      const uint4* srcv = (const uint4*)yt;
      for (int e = tid; e < Ny * ldm / 16; e += kThreads) dst[e] = srcv[e];
      __syncthreads();
    }
    int flip = 0;
    auto eps_at = [&](double b) {
      if (Ny <= 64) {
        flip ^= 1;
        return yl ? eval_eps_narrow<true>(b, Mc, Ny, ldm, dm0, dmin, (const uint8_t*)L.winp, y0v, hs,
                                          flip)
                  : eval_eps_narrow<false>(b, Mc, Ny, ldm, dm0, dmin, yt, y0v, hs, flip);
      }
      return yl ? eval_eps<true>(b, Mc, Ny, B2, ldm, dm0, dmin, ew, (const uint8_t*)L.winp, nullptr,
                                 y0v, ytil, nullptr, hs)
                : eval_eps<false>(b, Mc, Ny, B2, ldm, dm0, dmin, ew, yt, nullptr, y0v, ytil, nullptr,
                                  hs);
    };

    if (Ny <= 32) {
      if (tid < 33) hs.ginv[tid] = 1.0 / (2.0 * (D0 * exp2((double)(tid - 8) / 2.0)));
      __syncthreads();
      if (yl)
        grid_eps_narrow<true>(Mc, Ny, ldm, dm0, dmin, (const uint8_t*)L.winp, y0v, hs);
      else
        grid_eps_narrow<false>(Mc, Ny, ldm, dm0, dmin, yt, y0v, hs);
    } else if (Ny <= kGridPassNy)
      for (int g = 0; g < 33; ++g) {
        const double e = eps_at(D0 * exp2((double)(g - 8) / 2.0));
        if (tid == 0) hs.eg[g] = e;
      }
    __syncthreads();
    double emin = INFINITY;
    for (int g = 0; g < 33; ++g) emin = fmin(emin, hs.eg[g]);

    // -- beta: first grid minimiser, golden-section refinement on log beta
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
      double fc = eps_at(exp(ct));
      double fd = eps_at(exp(dt));
      for (int it = 0; it < 40; ++it) {
        if (fc <= fd) {
          bt = dt; dt = ct; fd = fc;
          ct = bt - invphi * (bt - at);
          fc = eps_at(exp(ct));
        } else {
          at = ct; ct = dt; fc = fd;
          dt = at + invphi * (bt - at);
          fd = eps_at(exp(dt));
        }
      }
      beta = exp(0.5 * (at + bt));
      const double eb = eps_at(beta);
      if (!(eb < best_eps * (1.0 - kEpsTieRel))) beta = D0 * exp2((double)gstar / 2.0);
    }

    // -- I0: the min(Ny + 1, Mc) candidates of smallest (distance, index):
    //    the k0-th smallest packed key by radix selection (8 bits a pass,
    //    exact integer counts), then the keys up to it listed in candidate
    //    order (hql_partial: of smallest d / n, as floor(d 2^20 / n), which
    //    keeps the order of the fractions: distinct ones differ by
    //    >= 2^20 / n^2 > 3).  The keys live in the weight array, free here.
    const int k0 = min(Ny + 1, Mc);
    {
      __attribute__((address_space(3))) long long* keys =
          (__attribute__((address_space(3))) long long*)ew;
      for (int j = tid; j < Mc; j += kThreads) {
        const long long d = compd[j];
        keys[j] = (hp ? (d << 20) / cnl[j] : d) << 13 | j;
      }
      long long prefix = 0;                 // the key's bits above `shift` found so far
      int rank = k0;                        // its rank among the keys with that prefix
      for (int shift = hp ? 56 : 32; shift >= 0; shift -= 8) {
        hs.hist[tid] = 0;                   // kThreads == 256 bins
        __syncthreads();
        const long long hmask = shift + 8 >= 64 ? 0ll : ~((1ll << (shift + 8)) - 1);
        for (int j = tid; j < Mc; j += kThreads) {
          const long long k = keys[j];
          if (((k ^ prefix) & hmask) == 0) atomicAdd(&hs.hist[(int)((k >> shift) & 255)], 1);
        }
        __syncthreads();
        if (wave == 0) {
          int c4[4], sum4 = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) sum4 += (c4[q] = hs.hist[4 * lane + q]);
          int before = wave_incl_scan(sum4) - sum4;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (before < rank && before + c4[q] >= rank) {
              hs.pref = prefix | ((long long)(4 * lane + q) << shift);
              hs.rank = rank - before;
            }
            before += c4[q];
          }
        }
        __syncthreads();
        prefix = hs.pref;
        rank = hs.rank;
      }
      const long long lo = prefix;
      const int per = (Mc + kThreads - 1) / kThreads;
      const int j0 = min(Mc, tid * per), j1 = min(Mc, j0 + per);
      int cnt = 0;
      for (int j = j0; j < j1; ++j) cnt += keys[j] <= lo;
      int tot = 0;
      int pos = block_excl_scan(cnt, sh.scan, &tot);
      for (int j = j0; j < j1; ++j)
        if (keys[j] <= lo) i0l[pos++] = j;
      __syncthreads();
    }

    // -- leave-one-out predictions of the I0 members, 64 at a time
    double num = 0.0, den = 0.0;
    const double inv2b = 1.0 / (2.0 * beta);
    const int nd = B2 + Ny;
    for (int c0 = 0; c0 < k0; c0 += 64) {
      const int nc = min(64, k0 - c0);
      // (a) logits -D(y_i, y_j) / (2 beta), D from whitened dot products
      if (Ny <= kNarrowNy) {
        // a thread per candidate; the members' whitened rows in LDS
        if (Ny <= 32) logits_narrow<32>(V, i0l, c0, nc, NRs, Ny, vn, Mc, dch, inv2b, tl);
        else logits_narrow<kNarrowNy>(V, i0l, c0, nc, NRs, Ny, vn, Mc, dch, inv2b, tl);
      } else {
        gemm_f64<true, true>(
            nc, Mc, [=](int c, int k) { return glb(V)[(size_t)glb(i0l)[c0 + c] * NRs + k]; },
            [=](int k, int j) { return glb(V)[(size_t)j * NRs + k]; },
            [=](int, int, int& kb_, int& ke_) { kb_ = 0; ke_ = Ny; return true; },
            [=](int c, int j, double g) {
              const int ii = glb(i0l)[c0 + c];
              glb(dch)[(size_t)c * Mc + j] =
                  (j == ii) ? -INFINITY : -(glb(vn)[ii] + glb(vn)[j] - 2.0 * g) * inv2b;
            },
            tl);
      }
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
      const double* rowS = hs.rowS;
      // (c) residuals of the leave-one-out predictions, x_i - x~_i and
      //     y_i - y~_i, with z~_c = sum_j e_cj z_j / S_c over the dims of x
      //     (B2) and y (Ny)
      if (Ny <= kNarrowNy && nd <= kNarrowNd) {
        // a thread per output (c, dd); candidates staged 64 at a time
        lds_f64* es = (lds_f64*)tl;                                 // nc x 64 weights
        __attribute__((address_space(3))) uint8_t* zs =
            (__attribute__((address_space(3))) uint8_t*)(es + 64 * 64);   // nd x 68 bytes
        double acc[kNarrowOut];
#pragma unroll
        for (int t = 0; t < kNarrowOut; ++t) acc[t] = 0.0;
        for (int j0 = 0; j0 < Mc; j0 += 64) {
          for (int e = tid; e < nc * 64; e += kThreads) {
            const int c = e >> 6, jj = e & 63;
            es[e] = j0 + jj < Mc ? glb(dch)[(size_t)c * Mc + j0 + jj] : 0.0;
          }
          for (int e = tid; e < nd * 64; e += kThreads) {
            const int dd = e >> 6, jj = e & 63;
            zs[dd * 68 + jj] = dd < B2 ? glb(xt)[(size_t)dd * ldm + j0 + jj]
                                       : glb(yt)[(size_t)(dd - B2) * ldm + j0 + jj];
          }
          __syncthreads();
#pragma unroll
          for (int t = 0; t < kNarrowOut; ++t) {
            const int o = tid + kThreads * t;
            if (o < nc * nd) {
              const int c = o / nd, dd = o - c * nd;
              const lds_f64* er = es + c * 64;
              const __attribute__((address_space(3))) uint32_t* zr =
                  (const __attribute__((address_space(3))) uint32_t*)(zs + dd * 68);
              double a_ = acc[t];
              for (int q = 0; q < 16; ++q) {
                const uint32_t w = zr[q];
                a_ = fma(er[4 * q], (double)(w & 0xffu), a_);
                a_ = fma(er[4 * q + 1], (double)((w >> 8) & 0xffu), a_);
                a_ = fma(er[4 * q + 2], (double)((w >> 16) & 0xffu), a_);
                a_ = fma(er[4 * q + 3], (double)(w >> 24), a_);
              }
              acc[t] = a_;
            }
          }
          __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < kNarrowOut; ++t) {
          const int o = tid + kThreads * t;
          if (o < nc * nd) {
            const int c = o / nd, dd = o - c * nd;
            const int ii = glb(i0l)[c0 + c];
            const double own = dd < B2 ? (double)glb(xt)[(size_t)dd * ldm + ii]
                                       : (double)glb(yt)[(size_t)(dd - B2) * ldm + ii];
            glb(zch)[(size_t)c * ldz + dd] = own - acc[t] / ((const lds_f64*)rowS)[c];
          }
        }
        __syncthreads();
      } else {
        gemm_f64<true, true>(
            nc, nd, [=](int c, int j) { return glb(dch)[(size_t)c * Mc + j]; },
            [=](int j, int dd) {
              return dd < B2 ? (double)glb(xt)[(size_t)dd * ldm + j]
                             : (double)glb(yt)[(size_t)(dd - B2) * ldm + j];
            },
            [=](int, int, int& kb_, int& ke_) { kb_ = 0; ke_ = Mc; return true; },
            [=](int c, int dd, double v) {
              const int ii = glb(i0l)[c0 + c];
              const double own = dd < B2 ? (double)glb(xt)[(size_t)dd * ldm + ii]
                                         : (double)glb(yt)[(size_t)(dd - B2) * ldm + ii];
              glb(zch)[(size_t)c * ldz + dd] = own - v / ((const lds_f64*)rowS)[c];
            },
            tl);
      }
      // (d) c_i = A r_i; accumulate <c_i, x_i - x~_i> and ||c_i||^2
      gemm_f64<true, true>(
          nc, B2, [=](int c, int k) { return glb(zch)[(size_t)c * ldz + B2 + k]; },
          [=](int k, int q) { return glb(axy)[(size_t)q * NRs + k]; },
          [=](int, int, int& kb_, int& ke_) { kb_ = 0; ke_ = Ny; return true; },
          [=, &num, &den](int c, int q, double v) {
            num += v * glb(zch)[(size_t)c * ldz + q];
            den += v * v;
          },
          tl);
    }
    num = block_sum_d(num, hs.red);
    den = block_sum_d(den, hs.red);
    const double alpha = den > 0.0 ? num / den : 0.0;

    // -- x0_hat = x~(beta) + alpha A (y0 - y~(beta))
    eval_eps<false>(beta, Mc, Ny, B2, ldm, dm0, dmin, ew, yt, xt, y0v, ytil, xtil, hs);
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
  phase_tables(p, carve_main_lds(lds_raw, p), sh);
  for (int h = blockIdx.x; h < n_hql; h += gridDim.x)
    hql_block(a, p, ws, slot_bytes, st->round, h, h == (int)blockIdx.x, lds_raw, sh, hs, nullptr);
}

hipError_t launch_hql(const FrameArgs& a, const DevParams& p, unsigned char* ws, size_t slot_bytes,
                      int slots, hipStream_t s) {
  hipLaunchKernelGGL(k_hql, dim3(slots), dim3(kThreads), hql_lds_bytes(p), s, a, p, ws, slot_bytes);
  return hipGetLastError();
}

hipError_t set_hql_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_hql, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace skm
