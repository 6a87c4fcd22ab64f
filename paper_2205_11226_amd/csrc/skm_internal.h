// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "skmmse.h"

namespace skm {

constexpr int kThreads = 256;        // one workgroup = 4 wave64
constexpr int kMaxRadii = 16;
// candidates per thread in a contiguous slice: ceil(MC / kThreads) for the
// largest admissible window (W = 32, B = 4)
constexpr int kMaxPer = 17;
// frame slots in flight in skm_conceal_batch
constexpr int kMaxBatchStreams = 8;
constexpr int kMaxB = 16;
constexpr int kMaxRing = 8;
constexpr int kMaxWin = 32;
constexpr int kMaxWd = kMaxB + 2 * kMaxRing + 2 * kMaxWin;   // 96 window side
// elements of slack before and after the int16 value plane: window loads of
// the estimation kernels may touch up to 8 elements beyond either end
constexpr int kValGuard = 8;

// device error bits (RoundState::err)
constexpr int kPartialBit = 1 << 16;   // m0cnt flag: the block holds received pixels
constexpr int kErrPartial = 1;       // lost pixel outside the in-frame cells
constexpr int kErrNoContext = 2;     // pending blocks, none touches a known pixel
constexpr int kErrHqlPending = 4;    // a block needs HQL and no HQL pass ran

struct DevParams {
  int B, r, W;
  int Wd;          // window side B + 2r + 2W
  int Wp;          // LDS row pitch of the window, Wd | 1: with an odd pitch the
                   // candidates of one window column fall into distinct banks
  int F;           // footprint side B + 2r
  int ND;          // (2W+1)^2 displacements
  int NR;          // ring pixels F^2 - B^2
  int MC;          // bound on admissible candidates
  int nrad;
  int radii[kMaxRadii];
  // expansion bucket of each Chebyshev radius rho <= W (4 bits per rho: the
  // first schedule radius >= rho), word rho / 16
  unsigned long long bucket_lut[3];
  int min_pct, min_hql, mode;
  int hql_partial; // HQL over every admissible candidate (partly known contexts completed)
  int prep_grid;   // workgroups of the round preparation (prep kernel, or the gate in CNN mode)
  int cnn_active;  // CNN mode with a loaded network (else the profile rule)
  int width, height, stride;
  int gh, gw;      // full cells
  double sigma2, t_phi, log_tnu, ridge_rel;
};

struct RoundState {
  int n_lost;
  int remaining;       // pending blocks at the start of the current round
  int round;           // current round, 1-based
  int err;
  int n_hql;           // blocks of this round waiting for the HQL kernel
  unsigned long long n_avail;     // fill: known pixels and their sum
  unsigned long long sum_avail;
  // Context rule of the round, from the prep or gate workgroups: ctx_nq is 1
  // when some pending block has |m0| >= r B, ctx_max the largest |m0| of the
  // workgroups without one; zeroed where a round starts (k_init,
  // k_round_finalize).  See note_context_rule.
  int ctx_nq;
  int ctx_max;
  // Zero between launches (the slot's allocation starts zeroed; the kernel
  // that consumes a field clears it):
  int err_geo;                    // geometry errors found by k_init
  unsigned int ticket;            // k_init workgroups done (the last one clears it)
  unsigned long long round_acc;   // end-of-round counts and ticket (k_round_finalize)
};

constexpr int kPrepGridMax = 512;   // workgroups of the prep kernel

// bstate values: 0 pending, > 0 concealed in that round, kNeedHql + round:
// waiting for the HQL kernels in that round.
constexpr int kNeedHql = 1 << 20;

struct FrameArgs {
  const uint8_t* frame;
  const uint8_t* mask;
  uint8_t* work;          // output plane (caller's out), same stride
  int16_t* val;           // workspace plane, pitch = width: pixel value where
                          // known (received or concealed in an earlier round),
                          // -1 where still lost
  unsigned int* cellbits; // lost-cell bit table, ceil(gh * gw / 32) words, zero between frames
  int* blk;               // lost cell indices, raster order
  int* bstate;
  int* m0cnt;             // known in-frame context pixels of each pending block
                          // (ring and the block's own), | kPartialBit when
                          // the block holds received pixels
  int2* ring;             // their sum, and min | max << 16 (prep kernel)
  int* hql_list;          // lost-block indices waiting for HQL in this round
  int8_t* gate;           // CNN mode: layer chosen for each lost block
  float* gate_pred;       // CNN mode: the two predicted gains of each lost block
  RoundState* st;
  RoundState* hstate;     // host-visible copy, written when a step publishes the state
  skm_block_info* info;   // optional
  float* xhat;            // optional
  int* dist;              // optional distance table (parity entry point)
  int* cnt;
  int cap;                // capacity of info / xhat in blocks
};

// ------------------------------------------------------------ batching
// Frames of equal size and parameters are concealed together: every stage of
// the pipeline is one launch over the (frame, lost block) items of all of
// them, with per-frame state as in the single-frame pipeline.  The frames'
// workspaces are equal slices of one allocation, so frame f's FrameArgs are
// frame 0's plus f strides, with the caller's buffers from a table.
struct BatchState {
  int total;               // lost blocks of all frames (items), written by k_init_b
  int remaining;           // pending blocks of all frames at the start of the next round
  int err;                 // OR of the frames' error bits
  unsigned frames_done;    // k_init_b: frames listed so far (zero between launches)
  unsigned fin_ticket;     // k_round_finalize_b: workgroups done (zero between launches)
  int pending;             // blocks of the round left pending by the estimation kernel
                           // (context rule, or waiting for HQL until the HQL kernel
                           // takes them); zero between rounds
  int pad[2];
};

struct FrameIO {           // the caller's buffers of one frame
  const uint8_t* frame;
  const uint8_t* mask;
  uint8_t* out;
  skm_block_info* info;
  float* xhat;
  int cap;
  int pad;
};

struct BatchArgs {
  FrameArgs a0;            // frame 0's workspace (its caller buffers unused)
  size_t val_stride;       // int16 elements between consecutive value planes
  int cell_stride;         // entries between consecutive block tables
  int bits_stride;         // words between consecutive cell bit tables
  int nf;
  const FrameIO* io;       // [nf]
  int* cum;                // [nf + 1] lost blocks of the frames before f (k_init_b)
  BatchState* bs;
  BatchState* hbs;         // host-visible copy (pinned), written where bs is published
};

// FrameArgs of frame f of a batch
__host__ __device__ inline FrameArgs batch_frame(const BatchArgs& b, int f) {
  FrameArgs a = b.a0;
  a.val += (size_t)f * b.val_stride;
  a.cellbits += (size_t)f * b.bits_stride;
  const size_t c = (size_t)f * b.cell_stride;
  a.blk += c; a.bstate += c; a.m0cnt += c; a.ring += c; a.hql_list += c;
  a.gate += c; a.gate_pred += 2 * c;
  a.st += f;
  if (a.hstate) a.hstate += f;
  const FrameIO& io = b.io[f];
  a.frame = io.frame; a.mask = io.mask; a.work = io.out;
  a.info = io.info; a.xhat = io.xhat; a.cap = io.cap;
  return a;
}

// geometry workgroups of one frame (k_init grid)
__host__ __device__ inline int init_wg_x(const DevParams& p) { return (p.width + 4 * kThreads - 1) / (4 * kThreads); }
__host__ __device__ inline int init_wgs(const DevParams& p) { return init_wg_x(p) * ((p.height + p.B - 1) / p.B); }

// batched launchers (every frame has the parameters and size of p)
hipError_t launch_init_b(const BatchArgs& b, const DevParams& p, hipStream_t s);
hipError_t launch_prep_b(const BatchArgs& b, const DevParams& p, int grid, hipStream_t s);
hipError_t launch_est_b(const BatchArgs& b, const DevParams& p, int variant, hipStream_t s);
hipError_t launch_finalize_b(const BatchArgs& b, const DevParams& p, int grid, hipStream_t s);
hipError_t launch_cnn_gate_b(const BatchArgs& b, const DevParams& p, const uint4* pk,
                             const float* wq, float tau1, float tau2, int grid, hipStream_t s);
// estimation kernel variants for p's geometry (candidate slices per thread),
// the first being the default; returns the count written to out (<= 4)
int est_variants(const DevParams& p, int* out);

// launchers (skm_kernels.hip)
hipError_t launch_init(const FrameArgs& a, const DevParams& p, hipStream_t s);
hipError_t launch_prep(const FrameArgs& a, const DevParams& p, int max_blocks,
                       hipStream_t s);
hipError_t launch_est(const FrameArgs& a, const DevParams& p, int max_blocks, hipStream_t s);
hipError_t launch_finalize(const FrameArgs& a, const DevParams& p, int max_blocks,
                           hipStream_t s);
hipError_t launch_fill(const FrameArgs& a, const DevParams& p, int max_blocks,
                       hipStream_t s);
hipError_t launch_dist(const FrameArgs& a, const DevParams& p, int max_blocks,
                       hipStream_t s);
hipError_t set_main_lds_limit(size_t bytes);
// n 32-bit words at p set to zero by a fill kernel (no memset node)
hipError_t launch_zero_words(unsigned int* p, size_t n, hipStream_t s);
// CNN gate (skm_cnn.hip)
constexpr int kCnnParams = 20898;
struct CnnBuffers {
  float *z1, *a1, *z2, *a2, *z3, *a3, *g, *y, *gy, *gz3, *gz2, *gz1;
};
constexpr size_t kCnnFloatsPerSample = 2 * 32 * 144 + 2 * 32 * 36 + 2 * 32 * 9 + 32 + 2 + 2 +
                                       32 * 9 + 32 * 36 + 32 * 144;
hipError_t launch_cnn_inputs(const FrameArgs& a, const DevParams& p, uint16_t* out, int max_blocks,
                             hipStream_t s);
hipError_t launch_cnn_gate(const FrameArgs& a, const DevParams& p, const uint4* pk,
                           const float* wq, float tau1,
                           float tau2, int max_blocks, hipStream_t s);
hipError_t cnn_infer(const uint16_t* x, int n, const uint4* pk, const float* wq, float* y,
                     hipStream_t s);
// register images of the gate weights for the inference kernels (after every
// change of the rounded weights)
hipError_t cnn_pack(const float* wq, uint4* pk, hipStream_t s);
size_t cnn_pack_bytes();
int cnn_gate_grid(int requested);
size_t cnn_gate_lds_bytes();
hipError_t set_cnn_gate_lds_limit(size_t bytes);
hipError_t cnn_init(float* prm, float* wq, unsigned long long seed, hipStream_t s);
hipError_t cnn_quantize(const float* prm, float* wq, hipStream_t s);
hipError_t cnn_forward(const CnnBuffers& b, const float* wq, const uint16_t* x, int N, hipStream_t s);
hipError_t cnn_backward(const CnnBuffers& b, const float* wq, const uint16_t* x, const float* t,
                        int N, float* grad, float* loss, hipStream_t s);
hipError_t cnn_adam(float* prm, const float* grad, float* m, float* v, float* wq, float lr, int step,
                    hipStream_t s);

// HQL (skm_hql.hip)
// workgroups of the HQL kernel, one scratch slot each: as many as a 1 GiB
// scratch holds, within [kHqlSlots, kHqlSlotsMax] (128 for 16 x 16 blocks,
// whose slots take ~13 MB; ~1000 for 2 x 2 patches)
constexpr int kHqlSlots = 128;
constexpr int kHqlSlotsMax = 1024;
constexpr size_t kHqlScratchBudget = size_t(1) << 30;
size_t hql_slot_bytes(const DevParams& p);
int hql_slots(const DevParams& p);
size_t hql_lds_bytes(const DevParams& p);
hipError_t launch_hql(const FrameArgs& a, const DevParams& p, unsigned char* ws, size_t slot_bytes,
                      int slots, hipStream_t s);
hipError_t set_hql_lds_limit(size_t bytes);
int prep_grid_for(int max_blocks);
size_t main_lds_bytes(const DevParams& p);

}  // namespace skm
