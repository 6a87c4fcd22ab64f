// Host side of the C ABI declared in include/skmmse.h.
//
// A context owns frame slots.  A slot is the device workspace of one frame in
// flight (value plane, block tables, round state, gate and HQL scratch), a
// private stream and one cached executable hipGraph of the frame pipeline.
// Slot 0 serves the single-frame entry points; slots 1.. serve
// skm_conceal_batch, which keeps several frames in flight on their streams.
//
// The frame pipeline is: loss geometry (k_init; its last workgroup lists the
// lost cells), then rounds of ([prep | gate], estimation, [HQL], finalize)
// until no block is pending; the last workgroups of k_init and of each
// finalize write the round state into coherent pinned memory.  A frame is
// enqueued with R rounds (the count its slot needed last time; rounds past
// the last are no-ops on the device).  After the frame's stream is
// synchronised, more rounds are run if blocks are still pending.  The
// enqueued part is captured once into a hipGraph and replayed while the
// frame pointers, parameters and R stay the same.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "skm_internal.h"

using namespace skm;

struct FrameSlot {
  int16_t* d_val = nullptr;       size_t cap_px = 0;
  unsigned int* d_cellbits = nullptr;
  int* d_blk = nullptr;
  int* d_bstate = nullptr;
  int* d_m0cnt = nullptr;
  int2* d_ring = nullptr;
  int* d_hql_list = nullptr;      size_t cap_cells = 0;
  unsigned char* d_hql_ws = nullptr; size_t cap_hql = 0;
  int8_t* d_gate = nullptr;
  float* d_gate_pred = nullptr;   size_t cap_gate = 0;
  RoundState* d_state = nullptr;
  RoundState* h_state = nullptr;  // pinned
  hipStream_t stream = nullptr;   // private: graph capture and batch work
  int last_rounds = 1;
  // cached executable graph of (geometry + R rounds + state copy)
  std::vector<unsigned char> gkey;
  hipGraphExec_t gexec = nullptr;
  // kernel timing: event pairs around the estimation kernel, per round
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  // batch bookkeeping: the frame in flight on this slot
  int pending = -1;
  DevParams pp;
  FrameArgs pa;
  int max_rounds = 0;
  int rounds_enqueued = 0;
  // the allocation-free slot: no kernel timing (no events), and at most this
  // many HQL workgroups (0: no cap beyond the context's)
  bool timing_off = false;
  int hql_slot_cap = 0;
};

// Launch shape of the batched pipeline for one geometry (block, ring, window):
// estimation kernel variant (candidate slices per thread) and the gate's
// workgroup count.
struct TileConfig {
  int block, ring, window;
  int est_variant;
  int gate_grid;
  double batch_ms;     // the autotuner's best batch time (informational)
};

// A group of batch frames with equal size and parameters, concealed by the
// batched kernels: one launch per stage over the (frame, block) items of all
// its frames.  Its workspace holds nf equal per-frame slices.
struct GroupSlot {
  unsigned char* d_pool = nullptr; size_t cap_pool = 0;
  std::vector<size_t> layout_key;    // offsets of the last layout (re-zeroed on change)
  FrameIO* d_io = nullptr;
  FrameIO* h_io = nullptr;           // pinned staging of the caller-buffer table
  size_t cap_io = 0;
  int* d_cum = nullptr; size_t cap_cum = 0;
  BatchState* d_bs = nullptr;
  BatchState* h_bs = nullptr;        // pinned, coherent: published by the kernels
  RoundState* h_states = nullptr;    // pinned, coherent: per-frame states
  size_t cap_states = 0;
  unsigned char* d_hql_ws = nullptr; size_t cap_hql = 0;
  hipStream_t stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<unsigned char> gkey;
  int last_rounds = 1;
  // the group in flight
  bool pending = false;
  std::vector<int> frames;           // indices into the caller's frame list
  DevParams p;
  BatchArgs b;
  int max_rounds = 0;
  int rounds_enqueued = 0;
  int est_variant = 0, gate_grid = 1280;
  // kernel timing: event pairs around the batched estimation kernel
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
};

struct skm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // host-memory entry point, CNN calls
  int max_lds = 65536;
  size_t lds_limit_set = 65536;
  size_t hql_lds_set = 65536;
  bool gate_lds_set = false;
  std::vector<FrameSlot*> slots;  // [0] single-frame calls, [1..] batch
  // skm_conceal_device_noalloc: its buffers are carved from the device's
  // `scratch` array per call; only the pinned host copy of the round state
  // is its own (allocated by skm_create)
  FrameSlot* na = nullptr;
  unsigned char* scratch_dev = nullptr;   // this device's copy of `scratch`
  // staging for the host-memory entry point
  uint8_t* d_frame = nullptr;     size_t cap_frame = 0;
  uint8_t* d_mask = nullptr;      size_t cap_mask = 0;
  uint8_t* d_out = nullptr;       size_t cap_out = 0;
  skm_block_info* d_info = nullptr; size_t cap_info = 0;
  // learned gate
  float* d_cnn = nullptr;       // [5][kCnnParams]: master, bf16 copy, Adam m, Adam v, gradient
  uint4* d_gate_pack = nullptr; // register images of the bf16 copy for the inference kernels
  float* d_cnn_loss = nullptr;
  bool cnn_loaded = false;
  int cnn_step = 0;
  float tau1 = 0.0f, tau2 = 0.0f;
  float* d_cnn_buf = nullptr;   size_t cap_cnn_buf = 0;   // training activations
  // batched mode of skm_conceal_batch: group slots (workspace, stream, graph)
  std::vector<GroupSlot*> groups;
  // tuned tile shapes per (block, ring, window), from skm_autotune or a cache
  std::vector<TileConfig> tiles;
  // options
  bool use_graphs = true;
  int batch_mode = 1;             // 1: batched kernels per group; 0: frame pipelines
  int batch_streams = 4;
  int gate_grid = 1280;             // five gate workgroups per CU
  int hql_grid = 0;               // 0: hql_slots(p)
  int est_variant = -1;           // -1: tuned or default
  int group_split = 1;            // batched mode: a group's frames in this many sub-groups
  // kernel timing (skm_profile_*)
  bool prof = false;
  double prof_ms = 0.0;
  int prof_launches = 0;
};

// ------------------------------------------- allocation-free workspace
// Device workspace of skm_conceal_device_noalloc.  Each GPU the library runs
// on holds its own copy of this array until the process ends.  In host code
// the name is only a stand-in: the address of a device's copy comes from
// hipGetSymbolAddress with that device current (resolve_scratch, called by
// skm_create) and is kept per device; only that address reaches kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

skm_status fail(skm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

skm_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? SKM_ENOMEM : SKM_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define SKM_HIP(call, what)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

template <typename T>
skm_status grow(T** ptr, size_t* cap, size_t need, const char* what) {
  if (need <= *cap && *ptr) return SKM_OK;
  if (*ptr) { (void)hipFree(*ptr); *ptr = nullptr; *cap = 0; }
  size_t n = need < 1 ? 1 : need;
  SKM_HIP(hipMalloc((void**)ptr, n * sizeof(T)), what);
  *cap = n;
  return SKM_OK;
}

std::mutex g_scratch_mu;
std::vector<unsigned char*> g_scratch_dev;   // per device, resolved once

// Address of this device's copy of `scratch` (hip_device must be current).
skm_status resolve_scratch(int hip_device, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= hip_device) g_scratch_dev.resize(hip_device + 1, nullptr);
  if (!g_scratch_dev[hip_device]) {
    void* ptr = nullptr;
    SKM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(SKM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[hip_device] = (unsigned char*)ptr;
  }
  *out = g_scratch_dev[hip_device];
  return SKM_OK;
}

bool mode_uses_hql(int mode) {
  return mode == SKM_MODE_PROFILE || mode == SKM_MODE_FULL || mode == SKM_MODE_CNN;
}

skm_status make_params(const skm_params* in, int width, int height, int stride, DevParams* p) {
  if (!in) return fail(SKM_EINVAL, "params is NULL");
  if (width <= 0 || height <= 0) return fail(SKM_EINVAL, "width and height must be positive");
  if (stride < width) return fail(SKM_EINVAL, "stride must be >= width");
  if (!(in->block == 2 || in->block == 4 || in->block == 8 || in->block == 16))
    return fail(SKM_EINVAL, "block must be 2, 4, 8 or 16");
  if (in->block == 2 && in->mode == SKM_MODE_CNN)
    return fail(SKM_EINVAL, "cnn mode needs block 4, 8 or 16");
  if (in->ring < 1 || in->ring > kMaxRing) return fail(SKM_EINVAL, "ring must be in 1..8");
  if (in->window < 1 || in->window > kMaxWin) return fail(SKM_EINVAL, "window must be in 1..32");
  if (in->expand_step < 1) return fail(SKM_EINVAL, "expand_step must be >= 1");
  if (in->min_overlap_pct < 0 || in->min_overlap_pct > 100)
    return fail(SKM_EINVAL, "min_overlap_pct must be in 0..100");
  if (in->min_hql_cands < 2) return fail(SKM_EINVAL, "min_hql_cands must be >= 2");
  if (in->mode < SKM_MODE_PROFILE || in->mode > SKM_MODE_PLAIN)
    return fail(SKM_EINVAL, "unknown mode");
  if (in->max_rounds < 0) return fail(SKM_EINVAL, "max_rounds must be >= 0");
  if (!(in->sigma2 > 0.0) || !isfinite(in->sigma2)) return fail(SKM_EINVAL, "sigma2 must be > 0");
  if (isnan(in->t_phi)) return fail(SKM_EINVAL, "t_phi is NaN");
  if (isnan(in->t_nu) || in->t_nu < 0.0) return fail(SKM_EINVAL, "t_nu must be >= 0");
  if (!(in->ridge_rel >= -1.0) || !isfinite(in->ridge_rel))
    return fail(SKM_EINVAL, "ridge_rel must be finite and >= -1");
  if (in->hql_partial != 0 && in->hql_partial != 1)
    return fail(SKM_EINVAL, "hql_partial must be 0 or 1");
  if (in->reserved != 0) return fail(SKM_EINVAL, "reserved must be 0");
  memset(p, 0, sizeof(*p));
  p->B = in->block; p->r = in->ring; p->W = in->window;
  p->Wd = p->B + 2 * p->r + 2 * p->W;
  p->Wp = p->Wd | 1;
  p->F = p->B + 2 * p->r;
  p->ND = (2 * p->W + 1) * (2 * p->W + 1);
  p->NR = p->F * p->F - p->B * p->B;
  {
    const int side = 2 * (p->B - 1 < p->W ? p->B - 1 : p->W) + 1;   // overlap the block itself
    p->MC = p->ND - side * side;
    if (p->MC < 1) p->MC = 1;
  }
  if (p->MC > kMaxPer * kThreads) return fail(SKM_EINVAL, "window too large for the block size");
  int n = 0;
  for (int rho = in->expand_step; rho < p->W; rho += in->expand_step) {
    if (n >= kMaxRadii - 1) return fail(SKM_EINVAL, "expand_step gives more than 16 radii");
    p->radii[n++] = rho;
  }
  p->radii[n++] = p->W;
  p->nrad = n;
  p->bucket_lut[0] = p->bucket_lut[1] = p->bucket_lut[2] = 0ull;
  for (int rho = 0; rho <= p->W; ++rho) {
    int b = n - 1;
    for (int ri = 0; ri < n; ++ri)
      if (p->radii[ri] >= rho) { b = ri; break; }
    p->bucket_lut[rho >> 4] |= (unsigned long long)b << (4 * (rho & 15));
  }
  p->hql_partial = in->hql_partial;
  p->min_pct = in->min_overlap_pct;
  p->min_hql = in->min_hql_cands;
  p->mode = in->mode;
  p->width = width; p->height = height; p->stride = stride;
  p->gh = height / p->B; p->gw = width / p->B;
  p->prep_grid = prep_grid_for(p->gh * p->gw);
  p->sigma2 = in->sigma2;
  p->t_phi = in->t_phi;
  p->log_tnu = in->t_nu > 0.0 ? log(in->t_nu) : -INFINITY;
  p->ridge_rel = in->ridge_rel;
  return SKM_OK;
}

skm_status slot_create(skm_ctx* c, FrameSlot** out) {
  FrameSlot* f = new (std::nothrow) FrameSlot();
  if (!f) return fail(SKM_ENOMEM, "slot allocation");
  *out = f;
  SKM_HIP(hipStreamCreateWithFlags(&f->stream, hipStreamNonBlocking), "hipStreamCreate");
  SKM_HIP(hipMalloc((void**)&f->d_state, sizeof(RoundState)), "round state");
  SKM_HIP(hipMemset(f->d_state, 0, sizeof(RoundState)), "round state");
  // coherent: kernels write the state here and the host reads it after a
  // stream synchronization
  SKM_HIP(hipHostMalloc((void**)&f->h_state, sizeof(RoundState), hipHostMallocCoherent),
          "pinned round state");
  memset(f->h_state, 0, sizeof(RoundState));
  (void)c;
  return SKM_OK;
}

void slot_destroy(FrameSlot* f) {
  if (!f) return;
  if (f->stream) (void)hipStreamSynchronize(f->stream);
  if (f->gexec) (void)hipGraphExecDestroy(f->gexec);
  (void)hipFree(f->d_val);
  (void)hipFree(f->d_cellbits);
  (void)hipFree(f->d_blk);
  (void)hipFree(f->d_bstate);
  (void)hipFree(f->d_m0cnt);
  (void)hipFree(f->d_ring);
  (void)hipFree(f->d_hql_list);
  (void)hipFree(f->d_hql_ws);
  (void)hipFree(f->d_gate);
  (void)hipFree(f->d_gate_pred);
  (void)hipFree(f->d_state);
  if (f->h_state) (void)hipHostFree(f->h_state);
  for (hipEvent_t e : f->ev) (void)hipEventDestroy(e);
  if (f->stream) (void)hipStreamDestroy(f->stream);
  delete f;
}

// The allocation-free slot of context c: this device's copy of `scratch`
// (resolved here, at set-up, with c's device current) and a pinned host copy
// of the round state.  Its device pointers are set per call.
skm_status na_create(skm_ctx* c) {
  skm_status s = resolve_scratch(c->device, &c->scratch_dev);
  if (s != SKM_OK) return s;
  FrameSlot* f = new (std::nothrow) FrameSlot();
  if (!f) return fail(SKM_ENOMEM, "slot allocation");
  c->na = f;
  f->timing_off = true;
  SKM_HIP(hipHostMalloc((void**)&f->h_state, sizeof(RoundState), hipHostMallocCoherent),
          "pinned round state");
  memset(f->h_state, 0, sizeof(RoundState));
  return SKM_OK;
}

// Dynamic LDS limits of the kernels for p's geometry (raised once, never
// lowered); fails if the device has too little LDS.
skm_status ensure_lds(skm_ctx* c, const DevParams& p) {
  if (!c->gate_lds_set) {
    SKM_HIP(set_cnn_gate_lds_limit(cnn_gate_lds_bytes()), "hipFuncSetAttribute");
    c->gate_lds_set = true;
  }
  if (mode_uses_hql(p.mode)) {
    const size_t hl = hql_lds_bytes(p);
    if ((int)hl > c->max_lds)
      return fail(SKM_EUNSUPPORTED, "window/ring/block need more LDS than the device has");
    if (hl > c->hql_lds_set) {
      SKM_HIP(set_hql_lds_limit(hl), "hipFuncSetAttribute");
      c->hql_lds_set = hl;
    }
  }
  size_t lds = main_lds_bytes(p);
  if ((int)lds > c->max_lds)
    return fail(SKM_EUNSUPPORTED, "window/ring/block need more LDS than the device has");
  if (lds > c->lds_limit_set) {
    SKM_HIP(set_main_lds_limit(lds), "hipFuncSetAttribute");
    c->lds_limit_set = lds;
  }
  return SKM_OK;
}

// Workspace of slot f for frames of p's geometry (grows, never shrinks), and
// the kernels' LDS limits.
skm_status ensure_frame(skm_ctx* c, FrameSlot* f, const DevParams& p) {
  size_t npx = (size_t)p.width * p.height;
  size_t ncell = (size_t)p.gh * p.gw;
  skm_status s;
  if ((s = grow(&f->d_val, &f->cap_px, npx + 2 * kValGuard, "workspace plane")) != SKM_OK)
    return s;
  if (ncell > f->cap_cells || !f->d_blk) {
    size_t cap = 0;
    (void)hipFree(f->d_cellbits); f->d_cellbits = nullptr;
    (void)hipFree(f->d_blk); f->d_blk = nullptr;
    (void)hipFree(f->d_bstate); f->d_bstate = nullptr;
    (void)hipFree(f->d_m0cnt); f->d_m0cnt = nullptr;
    (void)hipFree(f->d_ring); f->d_ring = nullptr;
    (void)hipFree(f->d_hql_list); f->d_hql_list = nullptr;
    f->cap_cells = 0;
    if ((s = grow(&f->d_cellbits, &cap, (ncell + 31) / 32, "cell table")) != SKM_OK) return s;
    SKM_HIP(hipMemset(f->d_cellbits, 0, sizeof(unsigned int) * cap), "cell table");
    cap = 0;
    if ((s = grow(&f->d_blk, &cap, ncell, "block list")) != SKM_OK) return s;
    cap = 0;
    if ((s = grow(&f->d_bstate, &cap, ncell, "block state")) != SKM_OK) return s;
    cap = 0;
    if ((s = grow(&f->d_m0cnt, &cap, ncell, "context counts")) != SKM_OK) return s;
    cap = 0;
    if ((s = grow(&f->d_ring, &cap, ncell, "context statistics")) != SKM_OK) return s;
    cap = 0;
    if ((s = grow(&f->d_hql_list, &cap, ncell, "HQL list")) != SKM_OK) return s;
    f->cap_cells = ncell < 1 ? 1 : ncell;
  }
  if (ncell > f->cap_gate || !f->d_gate) {
    (void)hipFree(f->d_gate); f->d_gate = nullptr;
    (void)hipFree(f->d_gate_pred); f->d_gate_pred = nullptr;
    const size_t n = ncell < 1 ? 1 : ncell;
    SKM_HIP(hipMalloc((void**)&f->d_gate, n), "gate");
    SKM_HIP(hipMalloc((void**)&f->d_gate_pred, sizeof(float) * 2 * n), "gate predictions");
    f->cap_gate = n;
  }
  if (mode_uses_hql(p.mode)) {
    const size_t need = hql_slot_bytes(p) * (size_t)hql_slots(p);
    if ((s = grow(&f->d_hql_ws, &f->cap_hql, need, "HQL scratch")) != SKM_OK) return s;
  }
  return ensure_lds(c, p);
}

FrameArgs frame_args(FrameSlot* f, const uint8_t* frame, const uint8_t* mask, uint8_t* out) {
  FrameArgs a;
  memset(&a, 0, sizeof(a));
  a.frame = frame; a.mask = mask; a.work = out;
  a.val = f->d_val + kValGuard; a.cellbits = f->d_cellbits; a.blk = f->d_blk;
  a.bstate = f->d_bstate; a.m0cnt = f->d_m0cnt; a.ring = f->d_ring;
  a.st = f->d_state;
  a.hstate = f->h_state;
  a.hql_list = f->d_hql_list;
  a.gate = f->d_gate; a.gate_pred = f->d_gate_pred;
  return a;
}

skm_status read_state(FrameSlot* f, hipStream_t s) {
  SKM_HIP(hipMemcpyAsync(f->h_state, f->d_state, sizeof(RoundState), hipMemcpyDeviceToHost, s),
          "state read-back");
  SKM_HIP(hipStreamSynchronize(s), "stream synchronize");
  return SKM_OK;
}

skm_status check_err(const RoundState& st) {
  if (st.err & kErrPartial)
    return fail(SKM_EUNSUPPORTED, "lost pixels must lie in the B x B cells inside the frame");
  if (st.err & kErrNoContext)
    return fail(SKM_EINVAL, "no lost block touches a received pixel (frame with no received pixel?)");
  if (st.err & kErrHqlPending)
    return fail(SKM_EUNSUPPORTED, "a block needs the HQL layer, which this build does not run");
  return SKM_OK;
}

// CNN mode with a loaded network: the gate kernel also prepares the round
// (ring statistics, per-workgroup context counts), in place of the prep kernel.
void activate_gate(const skm_ctx* c, DevParams& p) {
  p.cnn_active = p.mode == SKM_MODE_CNN && c->cnn_loaded;
  if (p.cnn_active) p.prep_grid = cnn_gate_grid(c->gate_grid);
}

// One round on s.  With timing on, the estimation kernel of round k of the
// enqueue is bracketed by event pair k of the slot.
skm_status launch_round(skm_ctx* c, FrameSlot* f, const DevParams& p, FrameArgs& a, int k,
                        hipStream_t s) {
  const int nb = p.gh * p.gw;
  if (p.cnn_active)
    SKM_HIP(launch_cnn_gate(a, p, c->d_gate_pack, c->d_cnn + kCnnParams, c->tau1, c->tau2,
                            c->gate_grid, s),
            "gate kernel");
  else
    SKM_HIP(launch_prep(a, p, nb, s), "prep kernel");
  const bool timed = c->prof && !f->timing_off;
  if (timed) {
    while ((int)f->ev.size() < 2 * (k + 1)) {
      hipEvent_t e;
      SKM_HIP(hipEventCreate(&e), "hipEventCreate");
      f->ev.push_back(e);
    }
    SKM_HIP(hipEventRecord(f->ev[2 * k], s), "hipEventRecord");
  }
  SKM_HIP(launch_est(a, p, nb, s), "estimation kernel");
  if (timed) SKM_HIP(hipEventRecord(f->ev[2 * k + 1], s), "hipEventRecord");
  if (mode_uses_hql(p.mode)) {
    int hg = c->hql_grid > 0 && c->hql_grid < hql_slots(p) ? c->hql_grid : hql_slots(p);
    if (f->hql_slot_cap > 0 && hg > f->hql_slot_cap) hg = f->hql_slot_cap;
    SKM_HIP(launch_hql(a, p, f->d_hql_ws, hql_slot_bytes(p), hg, s), "HQL kernel");
  }
  SKM_HIP(launch_finalize(a, p, nb, s), "finalize kernel");
  return SKM_OK;
}

// Geometry + R rounds, eagerly on s.
skm_status enqueue_eager(skm_ctx* c, FrameSlot* f, const DevParams& p, FrameArgs& a, int R,
                         hipStream_t s) {
  SKM_HIP(launch_init(a, p, s), "geometry kernels");
  for (int k = 0; k < R; ++k) {
    skm_status st = launch_round(c, f, p, a, k, s);
    if (st != SKM_OK) return st;
  }
  return SKM_OK;
}

// Enqueue a frame with R rounds on s: replay the slot's graph when its key
// (arguments, parameters, R, gate state, timing) matches, else capture one on
// the slot's private stream first.  Falls back to eager launches if graphs
// are off or capture fails.
skm_status enqueue_frame(skm_ctx* c, FrameSlot* f, const DevParams& p, FrameArgs& a, int R,
                         hipStream_t s) {
  f->ev_used = c->prof ? R : 0;
  f->rounds_enqueued = R;
  // with kernel timing on, launches are eager: the event pairs are read
  // back per frame, which this runtime does not allow for events recorded
  // by graph nodes
  if (!c->use_graphs || c->prof) return enqueue_eager(c, f, p, a, R, s);
  std::vector<unsigned char> key(sizeof(FrameArgs) + sizeof(DevParams) + 5 * sizeof(int) +
                                 2 * sizeof(float) + sizeof(void*));
  unsigned char* kp = key.data();
  memcpy(kp, &a, sizeof(FrameArgs)); kp += sizeof(FrameArgs);
  memcpy(kp, &p, sizeof(DevParams)); kp += sizeof(DevParams);
  const int ints[5] = {R, c->prof ? 1 : 0, c->gate_grid, (int)f->ev.size(), c->hql_grid};
  memcpy(kp, ints, sizeof(ints)); kp += sizeof(ints);
  memcpy(kp, &c->tau1, sizeof(float)); kp += sizeof(float);
  memcpy(kp, &c->tau2, sizeof(float)); kp += sizeof(float);
  memcpy(kp, &c->d_cnn, sizeof(void*));
  if (!f->gexec || key != f->gkey) {
    if (c->prof) {          // events must exist before capture
      while ((int)f->ev.size() < 2 * R) {
        hipEvent_t e;
        SKM_HIP(hipEventCreate(&e), "hipEventCreate");
        f->ev.push_back(e);
      }
      const int ev_n = (int)f->ev.size();
      memcpy(key.data() + sizeof(FrameArgs) + sizeof(DevParams) + 3 * sizeof(int), &ev_n,
             sizeof(int));
    }
    if (f->gexec) { (void)hipGraphExecDestroy(f->gexec); f->gexec = nullptr; }
    f->gkey.clear();
    hipGraph_t g = nullptr;
    SKM_HIP(hipStreamBeginCapture(f->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    skm_status st = enqueue_eager(c, f, p, a, R, f->stream);
    hipError_t e = hipStreamEndCapture(f->stream, &g);
    if (st != SKM_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      return st != SKM_OK ? st : hip_fail(e, "end capture");
    }
    e = hipGraphInstantiate(&f->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { f->gexec = nullptr; return hip_fail(e, "graph instantiate"); }
    f->gkey = key;
  }
  SKM_HIP(hipGraphLaunch(f->gexec, s), "graph launch");
  return SKM_OK;
}

// Wait for the frame enqueued on s, then run rounds until none is pending
// (or the round limit, then fill).  Reads kernel timing if it is on.
skm_status finish_frame(skm_ctx* c, FrameSlot* f, const DevParams& p, FrameArgs& a,
                        int max_rounds, hipStream_t s, int* n_lost_out, int* rounds_out) {
  SKM_HIP(hipStreamSynchronize(s), "stream synchronize");
  auto take_timing = [&]() -> skm_status {
    for (int k = 0; k < f->ev_used; ++k) {
      float ms = 0.f;
      SKM_HIP(hipEventElapsedTime(&ms, f->ev[2 * k], f->ev[2 * k + 1]), "hipEventElapsedTime");
      c->prof_ms += ms;
      ++c->prof_launches;
    }
    f->ev_used = 0;
    return SKM_OK;
  };
  skm_status st;
  if ((st = take_timing()) != SKM_OK) return st;
  if ((st = check_err(*f->h_state)) != SKM_OK) return st;
  int done = f->rounds_enqueued;
  int batch = done;
  while (f->h_state->remaining != 0) {
    if (max_rounds && done >= max_rounds) {
      SKM_HIP(launch_fill(a, p, p.gh * p.gw, s), "fill kernels");
      if ((st = read_state(f, s)) != SKM_OK) return st;
      break;
    }
    batch *= 2;
    if (max_rounds && batch > max_rounds - done) batch = max_rounds - done;
    f->ev_used = c->prof && !f->timing_off ? batch : 0;
    for (int k = 0; k < batch; ++k)
      if ((st = launch_round(c, f, p, a, k, s)) != SKM_OK) return st;
    done += batch;
    if ((st = read_state(f, s)) != SKM_OK) return st;
    if ((st = take_timing()) != SKM_OK) return st;
    if ((st = check_err(*f->h_state)) != SKM_OK) return st;
  }
  const int used = f->h_state->round - 1;
  f->last_rounds = used < 1 ? 1 : (used > 64 ? 64 : used);
  if (n_lost_out) *n_lost_out = f->h_state->n_lost;
  if (rounds_out) *rounds_out = used;
  return SKM_OK;
}

int initial_rounds(const FrameSlot* f, int max_rounds) {
  int R = f->last_rounds < 1 ? 1 : f->last_rounds;
  if (max_rounds && R > max_rounds) R = max_rounds;
  return R;
}

// Whole-frame pipeline on s; the frame is complete when this returns SKM_OK.
skm_status run_frame(skm_ctx* c, FrameSlot* f, const DevParams& p, FrameArgs& a, int max_rounds,
                     hipStream_t s, int* n_lost_out) {
  skm_status st = enqueue_frame(c, f, p, a, initial_rounds(f, max_rounds), s);
  if (st != SKM_OK) return st;
  return finish_frame(c, f, p, a, max_rounds, s, n_lost_out, nullptr);
}

// ----------------------------------------------------------- batch groups

skm_status group_create(GroupSlot** out) {
  GroupSlot* g = new (std::nothrow) GroupSlot();
  if (!g) return fail(SKM_ENOMEM, "group allocation");
  *out = g;
  SKM_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking), "hipStreamCreate");
  SKM_HIP(hipMalloc((void**)&g->d_bs, sizeof(BatchState)), "batch state");
  SKM_HIP(hipMemset(g->d_bs, 0, sizeof(BatchState)), "batch state");
  SKM_HIP(hipHostMalloc((void**)&g->h_bs, sizeof(BatchState), hipHostMallocCoherent),
          "pinned batch state");
  memset(g->h_bs, 0, sizeof(BatchState));
  return SKM_OK;
}

void group_destroy(GroupSlot* g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  (void)hipFree(g->d_pool);
  (void)hipFree(g->d_io);
  (void)hipFree(g->d_cum);
  (void)hipFree(g->d_bs);
  (void)hipFree(g->d_hql_ws);
  for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
  if (g->h_io) (void)hipHostFree(g->h_io);
  if (g->h_bs) (void)hipHostFree(g->h_bs);
  if (g->h_states) (void)hipHostFree(g->h_states);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

// Per-frame slices of a group's workspace: nf copies of each table.
struct PoolLayout {
  size_t val_stride, bits_stride, cell_stride;
  size_t o_state, o_bits, o_val, o_blk, o_bst, o_m0, o_ring, o_hl, o_gate, o_gp, total;
};

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

PoolLayout pool_layout(const DevParams& p, int nf) {
  PoolLayout L;
  const size_t npx = (size_t)p.width * p.height;
  const size_t ncell = (size_t)p.gh * p.gw < 1 ? 1 : (size_t)p.gh * p.gw;
  L.val_stride = round_up(npx + 2 * kValGuard, 128);
  L.bits_stride = round_up((ncell + 31) / 32, 64);
  L.cell_stride = round_up(ncell, 64);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  const size_t n = (size_t)nf;
  L.o_state = take(sizeof(RoundState) * n);
  L.o_bits = take(sizeof(unsigned int) * L.bits_stride * n);
  L.o_val = take(sizeof(int16_t) * L.val_stride * n);
  L.o_blk = take(sizeof(int) * L.cell_stride * n);
  L.o_bst = take(sizeof(int) * L.cell_stride * n);
  L.o_m0 = take(sizeof(int) * L.cell_stride * n);
  L.o_ring = take(sizeof(int2) * L.cell_stride * n);
  L.o_hl = take(sizeof(int) * L.cell_stride * n);
  L.o_gate = take(L.cell_stride * n);
  L.o_gp = take(sizeof(float) * 2 * L.cell_stride * n);
  L.total = off;
  return L;
}

int group_hql_slots(const skm_ctx* c, const DevParams& p) {
  const int n = hql_slots(p);
  return c->hql_grid > 0 && c->hql_grid < n ? c->hql_grid : n;
}

// Workspace and batch arguments of group g for nf frames of p's geometry.
// The round states and cell tables (the front of the pool) must be zero
// between launches: they are cleared when the pool is new or its layout
// changed; the kernels leave them zero after every frame.
skm_status group_prepare(skm_ctx* c, GroupSlot* g, const DevParams& p, int nf) {
  const PoolLayout L = pool_layout(p, nf);
  skm_status s;
  bool fresh = false;
  if (L.total > g->cap_pool || !g->d_pool) {
    if ((s = grow(&g->d_pool, &g->cap_pool, L.total, "batch workspace")) != SKM_OK) return s;
    fresh = true;
  }
  const std::vector<size_t> key = {L.o_state, L.o_bits, L.o_val, L.bits_stride};
  if (fresh || key != g->layout_key) {
    SKM_HIP(launch_zero_words((unsigned int*)(g->d_pool + L.o_state),
                              (L.o_val - L.o_state) / sizeof(unsigned int), g->stream),
            "batch workspace clear");
    g->layout_key = key;
  }
  if ((size_t)nf > g->cap_io || !g->d_io) {
    (void)hipFree(g->d_io); g->d_io = nullptr;
    if (g->h_io) { (void)hipHostFree(g->h_io); g->h_io = nullptr; }
    g->cap_io = 0;
    SKM_HIP(hipMalloc((void**)&g->d_io, sizeof(FrameIO) * nf), "frame table");
    SKM_HIP(hipHostMalloc((void**)&g->h_io, sizeof(FrameIO) * nf, 0), "frame table staging");
    g->cap_io = nf;
  }
  if ((s = grow(&g->d_cum, &g->cap_cum, (size_t)nf + 1, "item offsets")) != SKM_OK) return s;
  if ((size_t)nf > g->cap_states || !g->h_states) {
    if (g->h_states) (void)hipHostFree(g->h_states);
    g->h_states = nullptr;
    g->cap_states = 0;
    SKM_HIP(hipHostMalloc((void**)&g->h_states, sizeof(RoundState) * nf, hipHostMallocCoherent),
            "pinned frame states");
    memset(g->h_states, 0, sizeof(RoundState) * nf);
    g->cap_states = nf;
  }
  if (mode_uses_hql(p.mode)) {
    const size_t need = hql_slot_bytes(p) * (size_t)hql_slots(p);
    if ((s = grow(&g->d_hql_ws, &g->cap_hql, need, "HQL scratch")) != SKM_OK) return s;
  }
  if ((s = ensure_lds(c, p)) != SKM_OK) return s;
  BatchArgs& b = g->b;
  memset(&b, 0, sizeof(b));
  unsigned char* pool = g->d_pool;
  FrameArgs& a0 = b.a0;
  a0.st = (RoundState*)(pool + L.o_state);
  a0.hstate = g->h_states;
  a0.cellbits = (unsigned int*)(pool + L.o_bits);
  a0.val = (int16_t*)(pool + L.o_val) + kValGuard;
  a0.blk = (int*)(pool + L.o_blk);
  a0.bstate = (int*)(pool + L.o_bst);
  a0.m0cnt = (int*)(pool + L.o_m0);
  a0.ring = (int2*)(pool + L.o_ring);
  a0.hql_list = (int*)(pool + L.o_hl);
  a0.gate = (int8_t*)(pool + L.o_gate);
  a0.gate_pred = (float*)(pool + L.o_gp);
  b.val_stride = L.val_stride;
  b.cell_stride = (int)L.cell_stride;
  b.bits_stride = (int)L.bits_stride;
  b.nf = nf;
  b.io = g->d_io;
  b.cum = g->d_cum;
  b.bs = g->d_bs;
  b.hbs = g->h_bs;
  g->p = p;
  return SKM_OK;
}

// FrameArgs of frame f of group g on the host (caller buffers from the
// staging table)
FrameArgs group_frame_host(const GroupSlot* g, int f) {
  FrameArgs a = g->b.a0;
  a.val += (size_t)f * g->b.val_stride;
  a.cellbits += (size_t)f * g->b.bits_stride;
  const size_t cs = (size_t)f * g->b.cell_stride;
  a.blk += cs; a.bstate += cs; a.m0cnt += cs; a.ring += cs; a.hql_list += cs;
  a.gate += cs; a.gate_pred += 2 * cs;
  a.st += f;
  a.hstate += f;
  const FrameIO& io = g->h_io[f];
  a.frame = io.frame; a.mask = io.mask; a.work = io.out;
  a.info = io.info; a.xhat = io.xhat; a.cap = io.cap;
  return a;
}

int group_prep_grid(const DevParams& p, int nf) {
  const long long waves = (long long)nf * p.gh * p.gw;
  long long g = (waves + 3) / 4;
  if (g > 2048) g = 2048;
  if (g < 8) g = 8;
  return (int)((g + 7) / 8 * 8);
}

int group_fin_grid(const DevParams& p, int nf) {
  long long g = ((long long)nf * p.gh * p.gw + 15) / 16;
  return (int)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

skm_status launch_round_b(skm_ctx* c, GroupSlot* g, hipStream_t s) {
  const DevParams& p = g->p;
  const BatchArgs& b = g->b;
  if (p.cnn_active)
    SKM_HIP(launch_cnn_gate_b(b, p, c->d_gate_pack, c->d_cnn + kCnnParams, c->tau1, c->tau2,
                              g->gate_grid, s),
            "batched gate kernel");
  else
    SKM_HIP(launch_prep_b(b, p, group_prep_grid(p, b.nf), s), "batched prep kernel");
  const int k = g->ev_used;
  if (c->prof) {
    while ((int)g->ev.size() < 2 * (k + 1)) {
      hipEvent_t e;
      SKM_HIP(hipEventCreate(&e), "hipEventCreate");
      g->ev.push_back(e);
    }
    SKM_HIP(hipEventRecord(g->ev[2 * k], s), "hipEventRecord");
  }
  SKM_HIP(launch_est_b(b, p, g->est_variant, s), "batched estimation kernel");
  if (c->prof) {
    SKM_HIP(hipEventRecord(g->ev[2 * k + 1], s), "hipEventRecord");
    g->ev_used = k + 1;
  }
  // HQL: the single-frame kernel once per frame, in frame order, on the
  // group's scratch slots (a frame without HQL blocks returns at once)
  if (mode_uses_hql(p.mode)) {
    const int hg = group_hql_slots(c, p);
    for (int f = 0; f < b.nf; ++f)
      SKM_HIP(launch_hql(group_frame_host(g, f), p, g->d_hql_ws, hql_slot_bytes(p), hg, s),
              "HQL kernel");
  }
  SKM_HIP(launch_finalize_b(b, p, group_fin_grid(p, b.nf), s), "batched finalize kernel");
  return SKM_OK;
}

skm_status group_enqueue_eager(skm_ctx* c, GroupSlot* g, int R, hipStream_t s) {
  SKM_HIP(launch_init_b(g->b, g->p, s), "batched geometry kernel");
  for (int k = 0; k < R; ++k) {
    skm_status st = launch_round_b(c, g, s);
    if (st != SKM_OK) return st;
  }
  return SKM_OK;
}

// Geometry + R rounds of group g on its stream, replayed from a captured
// graph while the launch arguments repeat (the kernels read the caller
// buffers from the frame table, uploaded before each launch).
skm_status group_enqueue(skm_ctx* c, GroupSlot* g, int R) {
  g->rounds_enqueued = R;
  SKM_HIP(hipMemcpyAsync(g->d_io, g->h_io, sizeof(FrameIO) * g->b.nf, hipMemcpyHostToDevice,
                         g->stream),
          "frame table upload");
  g->ev_used = 0;
  // with kernel timing on, launches are eager (events recorded by graph
  // nodes cannot be queried for elapsed time)
  if (!c->use_graphs || c->prof) return group_enqueue_eager(c, g, R, g->stream);
  // the HQL launches take each frame's caller buffers as arguments, so with
  // HQL the buffers are part of the key
  const size_t io_bytes = mode_uses_hql(g->p.mode) ? sizeof(FrameIO) * g->b.nf : 0;
  std::vector<unsigned char> key(sizeof(BatchArgs) + sizeof(DevParams) + 4 * sizeof(int) +
                                 2 * sizeof(float) + sizeof(void*) + io_bytes);
  unsigned char* kp = key.data();
  memcpy(kp, &g->b, sizeof(BatchArgs)); kp += sizeof(BatchArgs);
  memcpy(kp, &g->p, sizeof(DevParams)); kp += sizeof(DevParams);
  const int ints[4] = {R, g->gate_grid, g->est_variant, c->hql_grid};
  memcpy(kp, ints, sizeof(ints)); kp += sizeof(ints);
  memcpy(kp, &c->tau1, sizeof(float)); kp += sizeof(float);
  memcpy(kp, &c->tau2, sizeof(float)); kp += sizeof(float);
  memcpy(kp, &c->d_cnn, sizeof(void*)); kp += sizeof(void*);
  if (io_bytes) memcpy(kp, g->h_io, io_bytes);
  if (!g->gexec || key != g->gkey) {
    if (g->gexec) { (void)hipGraphExecDestroy(g->gexec); g->gexec = nullptr; }
    g->gkey.clear();
    hipGraph_t graph = nullptr;
    SKM_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    skm_status st = group_enqueue_eager(c, g, R, g->stream);
    hipError_t e = hipStreamEndCapture(g->stream, &graph);
    if (st != SKM_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return st != SKM_OK ? st : hip_fail(e, "end capture");
    }
    e = hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { g->gexec = nullptr; return hip_fail(e, "graph instantiate"); }
    g->gkey = key;
  }
  SKM_HIP(hipGraphLaunch(g->gexec, g->stream), "graph launch");
  return SKM_OK;
}

// Wait for group g, run more rounds while blocks are pending (up to the
// round limit, then fill per frame), and write every frame's results.
skm_status group_finish(skm_ctx* c, GroupSlot* g, skm_frame_desc* frames) {
  g->pending = false;
  hipStream_t s = g->stream;
  SKM_HIP(hipStreamSynchronize(s), "stream synchronize");
  auto take_timing = [&]() -> skm_status {
    for (int k = 0; k < g->ev_used; ++k) {
      float ms = 0.f;
      SKM_HIP(hipEventElapsedTime(&ms, g->ev[2 * k], g->ev[2 * k + 1]), "hipEventElapsedTime");
      c->prof_ms += ms;
      ++c->prof_launches;
    }
    g->ev_used = 0;
    return SKM_OK;
  };
  skm_status tst = take_timing();
  if (tst != SKM_OK) return tst;
  int done = g->rounds_enqueued, batch = done < 1 ? 1 : done;
  skm_status st;
  while (g->h_bs->remaining != 0 && !(g->max_rounds && done >= g->max_rounds)) {
    batch *= 2;
    if (g->max_rounds && batch > g->max_rounds - done) batch = g->max_rounds - done;
    for (int k = 0; k < batch; ++k)
      if ((st = launch_round_b(c, g, s)) != SKM_OK) return st;
    done += batch;
    SKM_HIP(hipStreamSynchronize(s), "stream synchronize");
    if ((st = take_timing()) != SKM_OK) return st;
  }
  const int nf = g->b.nf;
  if (g->h_bs->remaining != 0) {
    // round limit: context-mean fill of each frame still pending
    for (int f = 0; f < nf; ++f) {
      if (g->h_states[f].remaining == 0) continue;
      SKM_HIP(launch_fill(group_frame_host(g, f), g->p, g->p.gh * g->p.gw, s), "fill kernels");
    }
    SKM_HIP(hipStreamSynchronize(s), "stream synchronize");
  }
  skm_status first = SKM_OK;
  int used_max = 1;
  for (int f = 0; f < nf; ++f) {
    skm_frame_desc& d = frames[g->frames[f]];
    const RoundState& rs = g->h_states[f];
    d.n_lost = rs.n_lost;
    const int used = rs.round - 1;
    d.rounds = used;
    used_max = used > used_max ? used : used_max;
    skm_status fs = check_err(rs);
    if (fs == SKM_OK && (d.info || d.xhat) && rs.n_lost > d.cap)
      fs = fail(SKM_EINVAL, "info/xhat capacity smaller than the number of lost blocks");
    d.status = fs;
    if (fs != SKM_OK && first == SKM_OK) first = fs;
  }
  g->last_rounds = used_max > 64 ? 64 : used_max;
  return first;
}

const TileConfig* tile_for(const skm_ctx* c, const DevParams& p) {
  for (const TileConfig& t : c->tiles)
    if (t.block == p.B && t.ring == p.r && t.window == p.W) return &t;
  return nullptr;
}

// skm_conceal_batch in batched mode.
skm_status batch_groups_run(skm_ctx* c, skm_frame_desc* frames, int32_t n, hipStream_t caller) {
  skm_status first = SKM_OK;
  std::vector<DevParams> prm(n);
  std::vector<int> ok(n, 0);
  for (int k = 0; k < n; ++k) {
    skm_frame_desc& d = frames[k];
    d.status = SKM_OK; d.n_lost = 0; d.rounds = 0;
    skm_status s = SKM_OK;
    if (!d.frame || !d.mask || !d.out || !d.params)
      s = fail(SKM_EINVAL, "frame, mask, out and params are required");
    else if ((d.info || d.xhat) && d.cap < 0)
      s = fail(SKM_EINVAL, "cap must be >= 0");
    else if ((s = make_params(d.params, d.width, d.height, d.stride, &prm[k])) == SKM_OK)
      activate_gate(c, prm[k]);
    if (s != SKM_OK) {
      d.status = s;
      if (first == SKM_OK) first = s;
      continue;
    }
    ok[k] = 1;
  }
  // groups of equal parameters and size, in order of their first frame
  std::vector<std::vector<int>> groups;
  std::vector<int> gmax;
  for (int k = 0; k < n; ++k) {
    if (!ok[k]) continue;
    int gi = -1;
    for (size_t q = 0; q < groups.size(); ++q) {
      const int r = groups[q][0];
      if (memcmp(&prm[r], &prm[k], sizeof(DevParams)) == 0 &&
          frames[r].params->max_rounds == frames[k].params->max_rounds) { gi = (int)q; break; }
    }
    if (gi < 0) { groups.push_back({}); gi = (int)groups.size() - 1; }
    groups[gi].push_back(k);
  }
  // sub-groups of contiguous frames, so that the stages of one overlap those
  // of another on the group streams
  if (c->group_split > 1) {
    std::vector<std::vector<int>> split;
    for (const std::vector<int>& gr : groups) {
      const int parts = (int)gr.size() < c->group_split ? (int)gr.size() : c->group_split;
      const int per = ((int)gr.size() + parts - 1) / parts;
      for (size_t k0 = 0; k0 < gr.size(); k0 += per)
        split.emplace_back(gr.begin() + k0, gr.begin() + std::min(gr.size(), k0 + (size_t)per));
    }
    groups.swap(split);
  }
  const int S = (int)groups.size() < c->batch_streams ? (int)groups.size() : c->batch_streams;
  while ((int)c->groups.size() < S) {
    GroupSlot* g = nullptr;
    skm_status s = group_create(&g);
    if (g) c->groups.push_back(g);
    if (s != SKM_OK) return s;
  }
  // order the groups' work after the caller's earlier work
  hipEvent_t ready = nullptr;
  SKM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming), "hipEventCreate");
  hipError_t e = hipEventRecord(ready, caller);
  for (int k = 0; k < S && e == hipSuccess; ++k) e = hipStreamWaitEvent(c->groups[k]->stream, ready, 0);
  (void)hipEventDestroy(ready);
  if (e != hipSuccess) return hip_fail(e, "batch ordering");
  for (size_t q = 0; q < groups.size(); ++q) {
    GroupSlot* g = c->groups[q % S];
    skm_status s;
    if (g->pending && (s = group_finish(c, g, frames)) != SKM_OK && first == SKM_OK) first = s;
    const std::vector<int>& fr = groups[q];
    const DevParams& p = prm[fr[0]];
    if ((s = group_prepare(c, g, p, (int)fr.size())) != SKM_OK) {
      for (int k : fr) frames[k].status = s;
      if (first == SKM_OK) first = s;
      continue;
    }
    for (size_t j = 0; j < fr.size(); ++j) {
      const skm_frame_desc& d = frames[fr[j]];
      FrameIO& io = g->h_io[j];
      io.frame = d.frame; io.mask = d.mask; io.out = d.out;
      io.info = d.info; io.xhat = d.xhat;
      io.cap = (d.info || d.xhat) ? d.cap : 0;
      io.pad = 0;
    }
    g->frames = fr;
    g->max_rounds = frames[fr[0]].params->max_rounds;
    // launch shape: the tuned one of this geometry, else the options
    const TileConfig* t = tile_for(c, p);
    int variants[4];
    const int nv = est_variants(p, variants);
    int v = t ? t->est_variant : (c->est_variant >= 0 ? c->est_variant : variants[0]);
    bool valid = false;
    for (int k = 0; k < nv; ++k) valid = valid || variants[k] == v;
    g->est_variant = valid ? v : variants[0];
    g->gate_grid = t ? t->gate_grid : c->gate_grid;
    int R = g->last_rounds < 1 ? 1 : g->last_rounds;
    if (g->max_rounds && R > g->max_rounds) R = g->max_rounds;
    if ((s = group_enqueue(c, g, R)) != SKM_OK) {
      for (int k : fr) frames[k].status = s;
      if (first == SKM_OK) first = s;
      continue;
    }
    g->pending = true;
  }
  for (int k = 0; k < S; ++k) {
    GroupSlot* g = c->groups[k];
    skm_status s;
    if (g->pending && (s = group_finish(c, g, frames)) != SKM_OK && first == SKM_OK) first = s;
  }
  return first;
}

}  // namespace

// integer value of "key": in text [b, e), or false
static bool json_int(const std::string& t, size_t b, size_t e, const char* key, int* out) {
  const std::string k = std::string("\"") + key + "\"";
  const size_t at = t.find(k, b);
  if (at == std::string::npos || at >= e) return false;
  size_t q = t.find(':', at + k.size());
  if (q == std::string::npos || q >= e) return false;
  char* end = nullptr;
  const long v = strtol(t.c_str() + q + 1, &end, 10);
  if (end == t.c_str() + q + 1) return false;
  *out = (int)v;
  return true;
}

extern "C" {

void skm_default_params(skm_params* p) {
  if (!p) return;
  p->block = 16; p->ring = 4; p->window = 24; p->expand_step = 4;
  p->min_overlap_pct = 50; p->min_hql_cands = 64; p->mode = SKM_MODE_PROFILE;
  p->max_rounds = 0; p->sigma2 = 10.0; p->t_phi = 20.0; p->t_nu = 0.1; p->ridge_rel = 1e-3;
  p->hql_partial = 0; p->reserved = 0;
}

void skm_patch_params(skm_params* p) {
  if (!p) return;
  skm_default_params(p);
  p->block = 2; p->ring = 2;
}

const char* skm_last_error(void) { return g_err.c_str(); }

skm_status skm_create(int32_t hip_device, skm_ctx** out) {
  if (!out) return fail(SKM_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  SKM_HIP(hipGetDeviceCount(&n), "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= n) return fail(SKM_EINVAL, "no such HIP device");
  SKM_HIP(hipSetDevice(hip_device), "hipSetDevice");
  skm_ctx* c = new (std::nothrow) skm_ctx();
  if (!c) return fail(SKM_ENOMEM, "context allocation");
  c->device = hip_device;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) ==
          hipSuccess && lds > 0)
    c->max_lds = lds;
  hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    skm_destroy(c);
    return hip_fail(e, "context setup");
  }
  FrameSlot* f0 = nullptr;
  skm_status s = slot_create(c, &f0);
  if (f0) c->slots.push_back(f0);
  if (s == SKM_OK) s = na_create(c);
  if (s != SKM_OK) {
    skm_destroy(c);
    return s;
  }
  *out = c;
  return SKM_OK;
}

void skm_destroy(skm_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (FrameSlot* f : c->slots) slot_destroy(f);
  for (GroupSlot* g : c->groups) group_destroy(g);
  if (c->na) {   // its device buffers live in `scratch`
    if (c->na->h_state) (void)hipHostFree(c->na->h_state);
    delete c->na;
  }
  (void)hipFree(c->d_cnn);
  (void)hipFree(c->d_gate_pack);
  (void)hipFree(c->d_cnn_loss);
  (void)hipFree(c->d_cnn_buf);
  (void)hipFree(c->d_frame);
  (void)hipFree(c->d_mask);
  (void)hipFree(c->d_out);
  (void)hipFree(c->d_info);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

skm_status skm_set_option(skm_ctx* c, int32_t option, int64_t value) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  switch (option) {
    case SKM_OPT_GRAPHS:
      if (value != 0 && value != 1) return fail(SKM_EINVAL, "SKM_OPT_GRAPHS takes 0 or 1");
      c->use_graphs = value != 0;
      return SKM_OK;
    case SKM_OPT_BATCH_STREAMS:
      if (value < 1 || value > kMaxBatchStreams)
        return fail(SKM_EINVAL, "SKM_OPT_BATCH_STREAMS takes 1..8");
      c->batch_streams = (int)value;
      return SKM_OK;
    case SKM_OPT_GATE_GRID:
      if (value < 8 || value > 4096 || value % 8 != 0)
        return fail(SKM_EINVAL, "SKM_OPT_GATE_GRID takes a multiple of 8 in 8..4096");
      c->gate_grid = (int)value;
      c->tiles.clear();
      return SKM_OK;
    case SKM_OPT_HQL_GRID:
      if (value < 0 || value > kHqlSlotsMax)
        return fail(SKM_EINVAL, "SKM_OPT_HQL_GRID takes 0..1024");
      c->hql_grid = (int)value;
      return SKM_OK;
    case SKM_OPT_BATCH_MODE:
      if (value != 0 && value != 1) return fail(SKM_EINVAL, "SKM_OPT_BATCH_MODE takes 0 or 1");
      c->batch_mode = (int)value;
      return SKM_OK;
    case SKM_OPT_EST_VARIANT:
      if (value < -1 || value > 3) return fail(SKM_EINVAL, "SKM_OPT_EST_VARIANT takes -1..3");
      c->est_variant = (int)value;
      c->tiles.clear();
      return SKM_OK;
    case SKM_OPT_GROUP_SPLIT:
      if (value < 1 || value > kMaxBatchStreams)
        return fail(SKM_EINVAL, "SKM_OPT_GROUP_SPLIT takes 1..8");
      c->group_split = (int)value;
      return SKM_OK;
    default:
      return fail(SKM_EINVAL, "unknown option");
  }
}

skm_status skm_get_option(skm_ctx* c, int32_t option, int64_t* value) {
  if (!c || !value) return fail(SKM_EINVAL, "NULL argument");
  switch (option) {
    case SKM_OPT_GRAPHS: *value = c->use_graphs ? 1 : 0; return SKM_OK;
    case SKM_OPT_BATCH_STREAMS: *value = c->batch_streams; return SKM_OK;
    case SKM_OPT_GATE_GRID: *value = c->gate_grid; return SKM_OK;
    case SKM_OPT_HQL_GRID: *value = c->hql_grid; return SKM_OK;
    case SKM_OPT_BATCH_MODE: *value = c->batch_mode; return SKM_OK;
    case SKM_OPT_EST_VARIANT: *value = c->est_variant; return SKM_OK;
    case SKM_OPT_GROUP_SPLIT: *value = c->group_split; return SKM_OK;
    default: return fail(SKM_EINVAL, "unknown option");
  }
}

skm_status skm_conceal_device(skm_ctx* c, const uint8_t* d_frame, const uint8_t* d_mask,
                              int32_t width, int32_t height, int32_t stride,
                              const skm_params* params, uint8_t* d_out,
                              skm_block_info* d_info, float* d_xhat, int32_t cap,
                              int32_t* n_lost, void* hip_stream) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (!d_frame || !d_mask || !d_out) return fail(SKM_EINVAL, "frame, mask and out are required");
  if ((d_info || d_xhat) && cap < 0) return fail(SKM_EINVAL, "cap must be >= 0");
  DevParams p;
  skm_status s = make_params(params, width, height, stride, &p);
  if (s != SKM_OK) return s;
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  FrameSlot* f = c->slots[0];
  if ((s = ensure_frame(c, f, p)) != SKM_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  activate_gate(c, p);
  FrameArgs a = frame_args(f, d_frame, d_mask, d_out);
  a.info = d_info; a.xhat = d_xhat; a.cap = (d_info || d_xhat) ? cap : 0;
  int nl = 0;
  if ((s = run_frame(c, f, p, a, params->max_rounds, st, &nl)) != SKM_OK) return s;
  if (n_lost) *n_lost = nl;
  if ((d_info || d_xhat) && nl > cap)
    return fail(SKM_EINVAL, "info/xhat capacity smaller than the number of lost blocks");
  return SKM_OK;
}

skm_status skm_conceal_device_noalloc(skm_ctx* c, const uint8_t* d_frame, const uint8_t* d_mask,
                                      int32_t width, int32_t height, int32_t stride,
                                      const skm_params* params, uint8_t* d_out,
                                      skm_block_info* d_info, float* d_xhat, int32_t cap,
                                      int32_t* n_lost, void* hip_stream) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (!d_frame || !d_mask || !d_out) return fail(SKM_EINVAL, "frame, mask and out are required");
  if ((d_info || d_xhat) && cap < 0) return fail(SKM_EINVAL, "cap must be >= 0");
  if (!c->na || !c->scratch_dev) return fail(SKM_EDEVICE, "allocation-free workspace not set up");
  DevParams p;
  skm_status s = make_params(params, width, height, stride, &p);
  if (s != SKM_OK) return s;
  // carve the frame's buffers out of this device's scratch copy
  const size_t npx = (size_t)p.width * p.height;
  const size_t ncell = (size_t)p.gh * p.gw < 1 ? 1 : (size_t)p.gh * p.gw;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  const size_t o_state = take(sizeof(RoundState));
  const size_t o_bits = take(sizeof(unsigned int) * ((ncell + 31) / 32));
  const size_t o_val = take(sizeof(int16_t) * (npx + 2 * kValGuard));
  const size_t o_blk = take(sizeof(int) * ncell);
  const size_t o_bst = take(sizeof(int) * ncell);
  const size_t o_m0 = take(sizeof(int) * ncell);
  const size_t o_ring = take(sizeof(int2) * ncell);
  const size_t o_hl = take(sizeof(int) * ncell);
  const size_t o_gate = take(ncell);
  const size_t o_gp = take(sizeof(float) * 2 * ncell);
  int hql_cap = 0;
  size_t o_hql = off;
  if (mode_uses_hql(p.mode)) {
    const size_t sb = hql_slot_bytes(p);
    const size_t room = off < kScratchBytes ? (kScratchBytes - off) / sb : 0;
    int want = c->hql_grid > 0 && c->hql_grid < hql_slots(p) ? c->hql_grid : hql_slots(p);
    hql_cap = room < (size_t)want ? (int)room : want;
    if (hql_cap < 1) off += sb;                 // report the size that one HQL slot needs
    else o_hql = take(sb * (size_t)hql_cap);
  }
  if (off > kScratchBytes) {
    char msg[200];
    snprintf(msg, sizeof msg,
             "frame needs %zu bytes of workspace; skm_conceal_device_noalloc has %zu "
             "(use skm_conceal_device)", off, kScratchBytes);
    return fail(SKM_EINVAL, msg);
  }
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  if ((s = ensure_lds(c, p)) != SKM_OK) return s;
  unsigned char* base = c->scratch_dev;
  FrameSlot* f = c->na;
  f->d_state = (RoundState*)(base + o_state);
  f->d_cellbits = (unsigned int*)(base + o_bits);
  f->d_val = (int16_t*)(base + o_val);
  f->d_blk = (int*)(base + o_blk);
  f->d_bstate = (int*)(base + o_bst);
  f->d_m0cnt = (int*)(base + o_m0);
  f->d_ring = (int2*)(base + o_ring);
  f->d_hql_list = (int*)(base + o_hl);
  f->d_gate = (int8_t*)(base + o_gate);
  f->d_gate_pred = (float*)(base + o_gp);
  f->d_hql_ws = hql_cap > 0 ? base + o_hql : nullptr;
  f->hql_slot_cap = hql_cap;
  hipStream_t st = (hipStream_t)hip_stream;
  // the array keeps the last call's contents: the round state and the cell
  // table start at zero (a fill kernel, no memset node)
  SKM_HIP(launch_zero_words((unsigned int*)(base + o_state),
                            (o_val - o_state) / sizeof(unsigned int), st),
          "workspace clear");
  activate_gate(c, p);
  FrameArgs a = frame_args(f, d_frame, d_mask, d_out);
  a.info = d_info; a.xhat = d_xhat; a.cap = (d_info || d_xhat) ? cap : 0;
  const int R = initial_rounds(f, params->max_rounds);
  f->ev_used = 0;
  f->rounds_enqueued = R;
  if ((s = enqueue_eager(c, f, p, a, R, st)) != SKM_OK) return s;
  int nl = 0;
  if ((s = finish_frame(c, f, p, a, params->max_rounds, st, &nl, nullptr)) != SKM_OK) return s;
  if (n_lost) *n_lost = nl;
  if ((d_info || d_xhat) && nl > cap)
    return fail(SKM_EINVAL, "info/xhat capacity smaller than the number of lost blocks");
  return SKM_OK;
}

skm_status skm_conceal(skm_ctx* c, const uint8_t* frame, const uint8_t* loss_mask,
                       int32_t width, int32_t height, int32_t stride,
                       const skm_params* params, uint8_t* out,
                       skm_block_info* info, int32_t info_cap, int32_t* n_lost) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (!frame || !loss_mask || !out) return fail(SKM_EINVAL, "frame, mask and out are required");
  if (info && info_cap < 0) return fail(SKM_EINVAL, "info_cap must be >= 0");
  DevParams p;
  skm_status s = make_params(params, width, height, stride, &p);
  if (s != SKM_OK) return s;
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  size_t bytes = (size_t)(height - 1) * stride + width;
  if ((s = grow(&c->d_frame, &c->cap_frame, bytes, "staging")) != SKM_OK) return s;
  if ((s = grow(&c->d_mask, &c->cap_mask, bytes, "staging")) != SKM_OK) return s;
  if ((s = grow(&c->d_out, &c->cap_out, bytes, "staging")) != SKM_OK) return s;
  int ncell = (width / params->block) * (height / params->block);
  if (info && (s = grow(&c->d_info, &c->cap_info, (size_t)(ncell < 1 ? 1 : ncell), "info")) != SKM_OK)
    return s;
  FrameSlot* f = c->slots[0];
  if ((s = ensure_frame(c, f, p)) != SKM_OK) return s;
  hipStream_t st = c->stream;
  activate_gate(c, p);
  SKM_HIP(hipMemcpyAsync(c->d_frame, frame, bytes, hipMemcpyHostToDevice, st), "frame upload");
  SKM_HIP(hipMemcpyAsync(c->d_mask, loss_mask, bytes, hipMemcpyHostToDevice, st), "mask upload");
  FrameArgs a = frame_args(f, c->d_frame, c->d_mask, c->d_out);
  a.info = info ? c->d_info : nullptr;
  a.cap = info ? ncell : 0;
  int nl = 0;
  if ((s = run_frame(c, f, p, a, params->max_rounds, st, &nl)) != SKM_OK) return s;
  if (n_lost) *n_lost = nl;
  if (info && nl > info_cap)
    return fail(SKM_EINVAL, "info_cap smaller than the number of lost blocks");
  SKM_HIP(hipMemcpyAsync(out, c->d_out, bytes, hipMemcpyDeviceToHost, st), "frame download");
  if (info && nl > 0)
    SKM_HIP(hipMemcpyAsync(info, c->d_info, sizeof(skm_block_info) * nl, hipMemcpyDeviceToHost, st),
            "info download");
  SKM_HIP(hipStreamSynchronize(st), "stream synchronize");
  return SKM_OK;
}

// ------------------------------------------------------------------ batch

static skm_status batch_finish(skm_ctx* c, FrameSlot* f, skm_frame_desc* frames) {
  skm_frame_desc& d = frames[f->pending];
  int nl = 0, rounds = 0;
  skm_status s = finish_frame(c, f, f->pp, f->pa, f->max_rounds, f->stream, &nl, &rounds);
  f->pending = -1;
  d.n_lost = nl;
  d.rounds = rounds;
  if (s == SKM_OK && (d.info || d.xhat) && nl > d.cap)
    s = fail(SKM_EINVAL, "info/xhat capacity smaller than the number of lost blocks");
  d.status = s;
  return s;
}

skm_status skm_conceal_batch(skm_ctx* c, skm_frame_desc* frames, int32_t n, void* hip_stream) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (n < 0 || (n > 0 && !frames)) return fail(SKM_EINVAL, "bad frame list");
  if (n == 0) return SKM_OK;
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  if (c->batch_mode == 1) return batch_groups_run(c, frames, n, (hipStream_t)hip_stream);
  const int S = n < c->batch_streams ? n : c->batch_streams;
  skm_status s;
  while ((int)c->slots.size() < 1 + S) {
    FrameSlot* f = nullptr;
    s = slot_create(c, &f);
    if (f) c->slots.push_back(f);
    if (s != SKM_OK) return s;
  }
  // order the batch after the caller's earlier work on hip_stream
  hipEvent_t ready = nullptr;
  SKM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming), "hipEventCreate");
  hipError_t e = hipEventRecord(ready, (hipStream_t)hip_stream);
  for (int k = 1; k <= S && e == hipSuccess; ++k) e = hipStreamWaitEvent(c->slots[k]->stream, ready, 0);
  (void)hipEventDestroy(ready);
  if (e != hipSuccess) return hip_fail(e, "batch ordering");
  skm_status first = SKM_OK;
  for (int k = 0; k < n; ++k) {
    skm_frame_desc& d = frames[k];
    d.status = SKM_OK; d.n_lost = 0; d.rounds = 0;
    FrameSlot* f = c->slots[1 + k % S];
    if (f->pending >= 0 && (s = batch_finish(c, f, frames)) != SKM_OK && first == SKM_OK) first = s;
    if (!d.frame || !d.mask || !d.out || !d.params) {
      d.status = fail(SKM_EINVAL, "frame, mask, out and params are required");
      if (first == SKM_OK) first = (skm_status)d.status;
      continue;
    }
    if ((d.info || d.xhat) && d.cap < 0) {
      d.status = fail(SKM_EINVAL, "cap must be >= 0");
      if (first == SKM_OK) first = (skm_status)d.status;
      continue;
    }
    DevParams p;
    if ((s = make_params(d.params, d.width, d.height, d.stride, &p)) == SKM_OK)
      s = ensure_frame(c, f, p);
    if (s != SKM_OK) {
      d.status = s;
      if (first == SKM_OK) first = s;
      continue;
    }
    activate_gate(c, p);
    f->pp = p;
    f->pa = frame_args(f, d.frame, d.mask, d.out);
    f->pa.info = d.info; f->pa.xhat = d.xhat; f->pa.cap = (d.info || d.xhat) ? d.cap : 0;
    f->max_rounds = d.params->max_rounds;
    if ((s = enqueue_frame(c, f, f->pp, f->pa, initial_rounds(f, f->max_rounds), f->stream)) != SKM_OK) {
      d.status = s;
      if (first == SKM_OK) first = s;
      continue;
    }
    f->pending = k;
  }
  for (int k = 1; k <= S; ++k) {
    FrameSlot* f = c->slots[k];
    if (f->pending >= 0 && (s = batch_finish(c, f, frames)) != SKM_OK && first == SKM_OK) first = s;
  }
  return first;
}

// Times the batch under each launch configuration and keeps the fastest:
// batched mode with every estimation variant of the first frame's geometry
// and gate grids 512, 768, 1536 and 3072 (CNN mode), graphs on and off; and
// frame pipelines on 1, 2, 4 or 8 streams with graphs on and off (gate grids
// 512, 768, 1536).  Each configuration: one warm call, then the best of
// `reps`.  The winner's batch mode, streams and graphs are set on the
// context; its estimation variant and gate grid are kept for the first
// frame's (block, ring, window) in the tile table.  The frames are concealed
// (several times) as a side effect.
skm_status skm_autotune(skm_ctx* c, skm_frame_desc* frames, int32_t n, int32_t reps,
                        double* best_ms) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (n < 1 || !frames || reps < 1 || !frames[0].params) return fail(SKM_EINVAL, "bad arguments");
  bool cnn = false;
  for (int k = 0; k < n; ++k) cnn = cnn || (frames[k].params && frames[k].params->mode == SKM_MODE_CNN);
  DevParams p0;
  skm_status s = make_params(frames[0].params, frames[0].width, frames[0].height, frames[0].stride,
                             &p0);
  if (s != SKM_OK) return s;
  int variants[4];
  const int nv = est_variants(p0, variants);
  const int grids_b[4] = {640, 1280, 2560, 3840};
  const int grids_s[3] = {640, 1280, 2560};
  const int streams[4] = {1, 2, 4, 8};
  const int splits[3] = {1, 2, 4};
  struct Cfg { int mode, streams, graphs, gate, variant, split; };
  std::vector<Cfg> cfgs;
  for (int graphs = 0; graphs <= 1; ++graphs) {
    for (int vi = 0; vi < nv; ++vi)
      for (int gi = 0; gi < (cnn ? 4 : 1); ++gi)
        for (int sp = 0; sp < 3; ++sp)
          if (splits[sp] == 1 || splits[sp] <= n)
            cfgs.push_back({1, 8, graphs, cnn ? grids_b[gi] : c->gate_grid, variants[vi],
                            splits[sp]});
    for (int si = 0; si < 4; ++si)
      for (int gi = 0; gi < (cnn ? 3 : 1); ++gi)
        cfgs.push_back({0, streams[si], graphs, cnn ? grids_s[gi] : c->gate_grid, -1, 1});
  }
  const int keep_mode = c->batch_mode, keep_streams = c->batch_streams;
  const bool keep_graphs = c->use_graphs;
  const int keep_gate = c->gate_grid, keep_var = c->est_variant, keep_split = c->group_split;
  std::vector<TileConfig> keep_tiles = c->tiles;
  c->tiles.clear();
  double best = 1e300;
  Cfg win = {keep_mode, keep_streams, keep_graphs ? 1 : 0, keep_gate, keep_var, keep_split};
  for (const Cfg& k : cfgs) {
    c->batch_mode = k.mode;
    c->batch_streams = k.streams;
    c->use_graphs = k.graphs != 0;
    c->gate_grid = k.gate;
    c->est_variant = k.variant;
    c->group_split = k.split;
    s = skm_conceal_batch(c, frames, n, nullptr);            // warm (captures graphs)
    if (s != SKM_OK) break;
    double t_best = 1e300;
    for (int r = 0; r < reps && s == SKM_OK; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      s = skm_conceal_batch(c, frames, n, nullptr);
      const double ms = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - t0).count();
      if (ms < t_best) t_best = ms;
    }
    if (s != SKM_OK) break;
    if (t_best < best) { best = t_best; win = k; }
  }
  c->tiles = keep_tiles;
  if (s != SKM_OK) {
    c->batch_mode = keep_mode; c->batch_streams = keep_streams; c->use_graphs = keep_graphs;
    c->gate_grid = keep_gate; c->est_variant = keep_var; c->group_split = keep_split;
    return s;
  }
  c->batch_mode = win.mode;
  c->batch_streams = win.mode == 1 ? keep_streams : win.streams;
  c->use_graphs = win.graphs != 0;
  c->est_variant = keep_var;
  c->group_split = win.mode == 1 ? win.split : keep_split;
  if (win.mode == 1) {
    c->gate_grid = keep_gate;
    TileConfig t = {p0.B, p0.r, p0.W, win.variant, win.gate, best};
    bool found = false;
    for (TileConfig& q : c->tiles)
      if (q.block == t.block && q.ring == t.ring && q.window == t.window) { q = t; found = true; }
    if (!found) c->tiles.push_back(t);
  } else {
    c->gate_grid = win.gate;
  }
  if (best_ms) *best_ms = best;
  return SKM_OK;
}

// Tuning cache: the context's launch options and tile table as JSON.
skm_status skm_autotune_save(skm_ctx* c, const char* path) {
  if (!c || !path) return fail(SKM_EINVAL, "NULL argument");
  FILE* fp = fopen(path, "w");
  if (!fp) return fail(SKM_EINVAL, std::string("cannot write ") + path);
  fprintf(fp, "{\n  \"version\": 1,\n  \"batch_mode\": %d,\n  \"batch_streams\": %d,\n"
              "  \"group_split\": %d,\n  \"graphs\": %d,\n  \"gate_grid\": %d,\n"
              "  \"tiles\": [",
          c->batch_mode, c->batch_streams, c->group_split, c->use_graphs ? 1 : 0, c->gate_grid);
  for (size_t k = 0; k < c->tiles.size(); ++k) {
    const TileConfig& t = c->tiles[k];
    fprintf(fp, "%s\n    {\"block\": %d, \"ring\": %d, \"window\": %d, \"est_variant\": %d, "
                "\"gate_grid\": %d, \"batch_ms\": %.6f}",
            k ? "," : "", t.block, t.ring, t.window, t.est_variant, t.gate_grid, t.batch_ms);
  }
  fprintf(fp, "\n  ]\n}\n");
  const bool bad = ferror(fp) != 0;
  fclose(fp);
  return bad ? fail(SKM_EINVAL, std::string("write error on ") + path) : SKM_OK;
}

skm_status skm_autotune_load(skm_ctx* c, const char* path) {
  if (!c || !path) return fail(SKM_EINVAL, "NULL argument");
  FILE* fp = fopen(path, "r");
  if (!fp) return fail(SKM_EINVAL, std::string("cannot read ") + path);
  std::string t;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, fp)) > 0) t.append(buf, got);
  fclose(fp);
  const size_t tiles_at = t.find("\"tiles\"");
  int version = 0, mode = 1, streams = 4, graphs = 1, gate = 768, split = 1;
  const size_t head_end = tiles_at == std::string::npos ? t.size() : tiles_at;
  if (!json_int(t, 0, head_end, "version", &version) || version != 1)
    return fail(SKM_EINVAL, "not a version-1 tuning file");
  if (!json_int(t, 0, head_end, "batch_mode", &mode) ||
      !json_int(t, 0, head_end, "batch_streams", &streams) ||
      !json_int(t, 0, head_end, "graphs", &graphs) || !json_int(t, 0, head_end, "gate_grid", &gate) ||
      !json_int(t, 0, head_end, "group_split", &split))
    return fail(SKM_EINVAL, "tuning file lacks a launch option");
  if ((mode != 0 && mode != 1) || streams < 1 || streams > kMaxBatchStreams ||
      split < 1 || split > kMaxBatchStreams ||
      (graphs != 0 && graphs != 1) || gate < 8 || gate > 4096 || gate % 8)
    return fail(SKM_EINVAL, "tuning file holds an out-of-range option");
  std::vector<TileConfig> tiles;
  if (tiles_at != std::string::npos) {
    size_t b = t.find('{', tiles_at);
    while (b != std::string::npos) {
      const size_t e = t.find('}', b);
      if (e == std::string::npos) return fail(SKM_EINVAL, "unterminated tile entry");
      TileConfig q = {0, 0, 0, 0, 0, 0.0};
      if (!json_int(t, b, e, "block", &q.block) || !json_int(t, b, e, "ring", &q.ring) ||
          !json_int(t, b, e, "window", &q.window) ||
          !json_int(t, b, e, "est_variant", &q.est_variant) ||
          !json_int(t, b, e, "gate_grid", &q.gate_grid))
        return fail(SKM_EINVAL, "tile entry lacks a field");
      if (q.est_variant < 0 || q.est_variant > 3 || q.gate_grid < 8 || q.gate_grid > 4096 ||
          q.gate_grid % 8)
        return fail(SKM_EINVAL, "tile entry out of range");
      tiles.push_back(q);
      b = t.find('{', e);
    }
  }
  c->batch_mode = mode;
  c->batch_streams = streams;
  c->group_split = split;
  c->use_graphs = graphs != 0;
  c->gate_grid = gate;
  c->tiles = tiles;
  return SKM_OK;
}

skm_status skm_distances_device(skm_ctx* c, const uint8_t* d_frame, const uint8_t* d_mask,
                                int32_t width, int32_t height, int32_t stride,
                                const skm_params* params, int32_t* d_dist, int32_t* d_cnt,
                                int32_t cap, int32_t* n_lost, void* hip_stream) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (!d_frame || !d_mask || !d_dist || !d_cnt) return fail(SKM_EINVAL, "NULL pointer");
  DevParams p;
  skm_status s = make_params(params, width, height, stride, &p);
  if (s != SKM_OK) return s;
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  FrameSlot* f = c->slots[0];
  if ((s = ensure_frame(c, f, p)) != SKM_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  size_t bytes = (size_t)(height - 1) * stride + width;
  if ((s = grow(&c->d_out, &c->cap_out, bytes, "scratch plane")) != SKM_OK) return s;
  FrameArgs a = frame_args(f, d_frame, d_mask, c->d_out);
  SKM_HIP(launch_init(a, p, st), "geometry kernels");
  if ((s = read_state(f, st)) != SKM_OK) return s;
  if ((s = check_err(*f->h_state)) != SKM_OK) return s;
  int nl = f->h_state->n_lost;
  if (n_lost) *n_lost = nl;
  if (nl > cap) return fail(SKM_EINVAL, "cap smaller than the number of lost blocks");
  a.dist = d_dist; a.cnt = d_cnt;
  SKM_HIP(launch_prep(a, p, p.gh * p.gw, st), "prep kernel");   // ring statistics
  SKM_HIP(launch_dist(a, p, p.gh * p.gw, st), "distance kernel");
  SKM_HIP(hipStreamSynchronize(st), "stream synchronize");
  return SKM_OK;
}

// ------------------------------------------------------------ learned gate

static skm_status cnn_params_alloc(skm_ctx* c) {
  if (c->d_cnn) return SKM_OK;
  SKM_HIP(hipMalloc((void**)&c->d_cnn, sizeof(float) * 5 * kCnnParams), "gate parameters");
  SKM_HIP(hipMemset(c->d_cnn, 0, sizeof(float) * 5 * kCnnParams), "gate parameters");
  SKM_HIP(hipMalloc((void**)&c->d_gate_pack, cnn_pack_bytes()), "packed gate weights");
  SKM_HIP(hipMalloc((void**)&c->d_cnn_loss, sizeof(float) * 4), "gate loss");
  return SKM_OK;
}

static skm_status cnn_buffers(skm_ctx* c, int n, CnnBuffers* b) {
  const size_t need = kCnnFloatsPerSample * (size_t)n;
  skm_status s = grow(&c->d_cnn_buf, &c->cap_cnn_buf, need, "gate activations");
  if (s != SKM_OK) return s;
  float* q = c->d_cnn_buf;
  auto take = [&](size_t per) { float* r = q; q += per * (size_t)n; return r; };
  b->z1 = take(32 * 144); b->a1 = take(32 * 144); b->z2 = take(32 * 36); b->a2 = take(32 * 36);
  b->z3 = take(32 * 9); b->a3 = take(32 * 9); b->g = take(32); b->y = take(2); b->gy = take(2);
  b->gz3 = take(32 * 9); b->gz2 = take(32 * 36); b->gz1 = take(32 * 144);
  return SKM_OK;
}

skm_status skm_cnn_init(skm_ctx* c, uint64_t seed) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  skm_status s = cnn_params_alloc(c);
  if (s != SKM_OK) return s;
  SKM_HIP(hipMemsetAsync(c->d_cnn + 2 * kCnnParams, 0, sizeof(float) * 2 * kCnnParams, c->stream),
          "Adam state");
  SKM_HIP(cnn_init(c->d_cnn, c->d_cnn + kCnnParams, seed, c->stream), "gate init");
  SKM_HIP(cnn_pack(c->d_cnn + kCnnParams, c->d_gate_pack, c->stream), "gate weight packing");
  SKM_HIP(hipStreamSynchronize(c->stream), "stream synchronize");
  c->cnn_step = 0;
  c->cnn_loaded = true;
  return SKM_OK;
}

skm_status skm_cnn_set_weights(skm_ctx* c, const float* host, int32_t n) {
  if (!c || !host) return fail(SKM_EINVAL, "NULL argument");
  if (n != kCnnParams) return fail(SKM_EINVAL, "weight count must be 20898");
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  skm_status s = cnn_params_alloc(c);
  if (s != SKM_OK) return s;
  SKM_HIP(hipMemcpyAsync(c->d_cnn, host, sizeof(float) * kCnnParams, hipMemcpyHostToDevice, c->stream),
          "weights upload");
  SKM_HIP(hipMemsetAsync(c->d_cnn + 2 * kCnnParams, 0, sizeof(float) * 2 * kCnnParams, c->stream),
          "Adam state");
  SKM_HIP(cnn_quantize(c->d_cnn, c->d_cnn + kCnnParams, c->stream), "quantize");
  SKM_HIP(cnn_pack(c->d_cnn + kCnnParams, c->d_gate_pack, c->stream), "gate weight packing");
  SKM_HIP(hipStreamSynchronize(c->stream), "stream synchronize");
  c->cnn_step = 0;
  c->cnn_loaded = true;
  return SKM_OK;
}

skm_status skm_cnn_get_weights(skm_ctx* c, float* host, int32_t n) {
  if (!c || !host) return fail(SKM_EINVAL, "NULL argument");
  if (n != kCnnParams) return fail(SKM_EINVAL, "weight count must be 20898");
  if (!c->cnn_loaded) return fail(SKM_EINVAL, "no network loaded");
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  SKM_HIP(hipMemcpyAsync(host, c->d_cnn, sizeof(float) * kCnnParams, hipMemcpyDeviceToHost, c->stream),
          "weights download");
  SKM_HIP(hipStreamSynchronize(c->stream), "stream synchronize");
  return SKM_OK;
}

skm_status skm_cnn_set_thresholds(skm_ctx* c, double tau1, double tau2) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (isnan(tau1) || isnan(tau2)) return fail(SKM_EINVAL, "threshold is NaN");
  c->tau1 = (float)tau1;
  c->tau2 = (float)tau2;
  return SKM_OK;
}

static const char kGateMagic[8] = {'S', 'K', 'M', 'G', 'A', 'T', 'E', '1'};
static const uint32_t kGateVersion = 2u;   // space-to-depth input, 20898 weights

skm_status skm_save_cnn(skm_ctx* c, const char* path) {
  if (!c || !path) return fail(SKM_EINVAL, "NULL argument");
  if (!c->cnn_loaded) return fail(SKM_EINVAL, "no network loaded");
  std::vector<float> w(kCnnParams);
  skm_status s = skm_cnn_get_weights(c, w.data(), kCnnParams);
  if (s != SKM_OK) return s;
  FILE* f = fopen(path, "wb");
  if (!f) return fail(SKM_EINVAL, std::string("cannot open ") + path);
  const uint32_t hdr[4] = {kGateVersion, (uint32_t)kCnnParams, 0u, 0u};
  const float tau[2] = {c->tau1, c->tau2};
  bool ok = fwrite(kGateMagic, 1, 8, f) == 8 && fwrite(hdr, 4, 4, f) == 4 &&
            fwrite(tau, 4, 2, f) == 2 && fwrite(w.data(), 4, kCnnParams, f) == (size_t)kCnnParams;
  ok = (fclose(f) == 0) && ok;
  return ok ? SKM_OK : fail(SKM_EINVAL, "write failed");
}

skm_status skm_load_cnn(skm_ctx* c, const char* path) {
  if (!c || !path) return fail(SKM_EINVAL, "NULL argument");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(SKM_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  uint32_t hdr[4];
  float tau[2];
  std::vector<float> w(kCnnParams);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kGateMagic, 8) == 0 &&
            fread(hdr, 4, 4, f) == 4 && hdr[0] == kGateVersion && hdr[1] == (uint32_t)kCnnParams &&
            fread(tau, 4, 2, f) == 2 && fread(w.data(), 4, kCnnParams, f) == (size_t)kCnnParams;
  fclose(f);
  if (!ok) return fail(SKM_EINVAL, "not a gate weight file (SKMGATE1, version 2, 20898 weights)");
  skm_status s = skm_cnn_set_weights(c, w.data(), kCnnParams);
  if (s != SKM_OK) return s;
  c->tau1 = tau[0];
  c->tau2 = tau[1];
  return SKM_OK;
}

skm_status skm_cnn_inputs(skm_ctx* c, const uint8_t* d_frame, const uint8_t* d_mask, int32_t width,
                          int32_t height, int32_t stride, const skm_params* params,
                          uint16_t* d_inputs, int32_t cap, int32_t* n_lost, void* hip_stream) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (!d_frame || !d_mask || !d_inputs) return fail(SKM_EINVAL, "NULL pointer");
  DevParams p;
  skm_status s = make_params(params, width, height, stride, &p);
  if (s != SKM_OK) return s;
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  if ((s = ensure_frame(c, c->slots[0], p)) != SKM_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t bytes = (size_t)(height - 1) * stride + width;
  if ((s = grow(&c->d_out, &c->cap_out, bytes, "scratch plane")) != SKM_OK) return s;
  FrameArgs a = frame_args(c->slots[0], d_frame, d_mask, c->d_out);
  SKM_HIP(launch_init(a, p, st), "geometry kernels");
  if ((s = read_state(c->slots[0], st)) != SKM_OK) return s;
  if ((s = check_err(*c->slots[0]->h_state)) != SKM_OK) return s;
  const int nl = c->slots[0]->h_state->n_lost;
  if (n_lost) *n_lost = nl;
  if (nl > cap) return fail(SKM_EINVAL, "cap smaller than the number of lost blocks");
  SKM_HIP(launch_cnn_inputs(a, p, d_inputs, p.gh * p.gw, st), "gate inputs");
  SKM_HIP(hipStreamSynchronize(st), "stream synchronize");
  return SKM_OK;
}

skm_status skm_cnn_forward(skm_ctx* c, const uint16_t* d_inputs, int32_t n, float* d_out,
                           void* hip_stream) {
  if (!c || !d_inputs || !d_out || n < 1) return fail(SKM_EINVAL, "bad argument");
  if (!c->cnn_loaded) return fail(SKM_EINVAL, "no network loaded");
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  if (!c->gate_lds_set) {
    SKM_HIP(set_cnn_gate_lds_limit(cnn_gate_lds_bytes()), "hipFuncSetAttribute");
    c->gate_lds_set = true;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  SKM_HIP(cnn_infer(d_inputs, n, c->d_gate_pack, c->d_cnn + kCnnParams, d_out, st),
          "gate inference");
  SKM_HIP(hipStreamSynchronize(st), "stream synchronize");
  return SKM_OK;
}

static skm_status cnn_fwd_bwd(skm_ctx* c, const uint16_t* x, const float* t, int n, hipStream_t st,
                              float* loss) {
  CnnBuffers b;
  skm_status s = cnn_buffers(c, n, &b);
  if (s != SKM_OK) return s;
  float* wq = c->d_cnn + kCnnParams;
  float* grad = c->d_cnn + 4 * kCnnParams;
  SKM_HIP(cnn_forward(b, wq, x, n, st), "gate forward");
  SKM_HIP(cnn_backward(b, wq, x, t, n, grad, c->d_cnn_loss, st), "gate backward");
  if (loss) {
    SKM_HIP(hipMemcpyAsync(loss, c->d_cnn_loss, sizeof(float), hipMemcpyDeviceToHost, st), "loss");
  }
  return SKM_OK;
}

skm_status skm_cnn_gradients(skm_ctx* c, const uint16_t* d_inputs, const float* d_targets, int32_t n,
                             float* host_grad, float* loss, void* hip_stream) {
  if (!c || !d_inputs || !d_targets || !host_grad || n < 1) return fail(SKM_EINVAL, "bad argument");
  if (!c->cnn_loaded) return fail(SKM_EINVAL, "no network loaded");
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)hip_stream;
  skm_status s = cnn_fwd_bwd(c, d_inputs, d_targets, n, st, loss);
  if (s != SKM_OK) return s;
  SKM_HIP(hipMemcpyAsync(host_grad, c->d_cnn + 4 * kCnnParams, sizeof(float) * kCnnParams,
                         hipMemcpyDeviceToHost, st), "gradient download");
  SKM_HIP(hipStreamSynchronize(st), "stream synchronize");
  return SKM_OK;
}

skm_status skm_cnn_train_step(skm_ctx* c, const uint16_t* d_inputs, const float* d_targets,
                              int32_t n, float lr, float* loss, void* hip_stream) {
  if (!c || !d_inputs || !d_targets || n < 1 || !(lr > 0.0f)) return fail(SKM_EINVAL, "bad argument");
  if (!c->cnn_loaded) return fail(SKM_EINVAL, "no network loaded");
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)hip_stream;
  skm_status s = cnn_fwd_bwd(c, d_inputs, d_targets, n, st, loss);
  if (s != SKM_OK) return s;
  ++c->cnn_step;
  SKM_HIP(cnn_adam(c->d_cnn, c->d_cnn + 4 * kCnnParams, c->d_cnn + 2 * kCnnParams,
                   c->d_cnn + 3 * kCnnParams, c->d_cnn + kCnnParams, lr, c->cnn_step, st), "Adam");
  SKM_HIP(cnn_pack(c->d_cnn + kCnnParams, c->d_gate_pack, st), "gate weight packing");
  if (loss) SKM_HIP(hipStreamSynchronize(st), "stream synchronize");
  return SKM_OK;
}

skm_status skm_cnn_last_predictions(skm_ctx* c, float* host, int32_t cap) {
  if (!c || !host) return fail(SKM_EINVAL, "NULL argument");
  if (!c->slots[0]->d_gate_pred) return fail(SKM_EINVAL, "no frame concealed yet");
  const size_t n = (size_t)cap < c->slots[0]->cap_gate ? (size_t)cap : c->slots[0]->cap_gate;
  SKM_HIP(hipSetDevice(c->device), "hipSetDevice");
  SKM_HIP(hipMemcpy(host, c->slots[0]->d_gate_pred, sizeof(float) * 2 * n, hipMemcpyDeviceToHost), "download");
  return SKM_OK;
}

skm_status skm_profile_enable(skm_ctx* c, int32_t enable) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  c->prof = enable != 0;
  return SKM_OK;
}

skm_status skm_profile_read(skm_ctx* c, double* total_ms, int32_t* launches) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (total_ms) *total_ms = c->prof_ms;
  if (launches) *launches = c->prof_launches;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  return SKM_OK;
}

}  // extern "C"
