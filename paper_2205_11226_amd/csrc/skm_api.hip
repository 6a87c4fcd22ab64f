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
  // options
  bool use_graphs = true;
  int batch_streams = 4;
  int gate_grid = 768;
  int hql_grid = 0;               // 0: hql_slots(p)
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
  memset(p, 0, sizeof(*p));
  p->B = in->block; p->r = in->ring; p->W = in->window;
  p->Wd = p->B + 2 * p->r + 2 * p->W;
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

}  // namespace

extern "C" {

void skm_default_params(skm_params* p) {
  if (!p) return;
  p->block = 16; p->ring = 4; p->window = 24; p->expand_step = 4;
  p->min_overlap_pct = 50; p->min_hql_cands = 64; p->mode = SKM_MODE_PROFILE;
  p->max_rounds = 0; p->sigma2 = 10.0; p->t_phi = 20.0; p->t_nu = 0.1; p->ridge_rel = 1e-3;
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
      return SKM_OK;
    case SKM_OPT_HQL_GRID:
      if (value < 0 || value > kHqlSlotsMax)
        return fail(SKM_EINVAL, "SKM_OPT_HQL_GRID takes 0..1024");
      c->hql_grid = (int)value;
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

// Times the batch under each launch configuration (streams 1, 2, 4, 8 with
// graphs on and off; gate grids 512, 768, 1536 in CNN mode), repeats `reps`
// times, keeps the fastest and reports its time.  The frames are concealed
// (several times) as a side effect.
skm_status skm_autotune(skm_ctx* c, skm_frame_desc* frames, int32_t n, int32_t reps,
                        double* best_ms) {
  if (!c) return fail(SKM_EINVAL, "ctx is NULL");
  if (n < 1 || !frames || reps < 1) return fail(SKM_EINVAL, "bad arguments");
  bool cnn = false;
  for (int k = 0; k < n; ++k) cnn = cnn || (frames[k].params && frames[k].params->mode == SKM_MODE_CNN);
  const int streams[4] = {1, 2, 4, 8};
  const int grids[3] = {512, 768, 1536};
  double best = 1e300;
  int bs = c->batch_streams, bg = c->use_graphs ? 1 : 0, bgg = c->gate_grid;
  for (int gi = 0; gi < (cnn ? 3 : 1); ++gi) {
    for (int graphs = 0; graphs <= 1; ++graphs) {
      for (int si = 0; si < 4; ++si) {
        c->batch_streams = streams[si];
        c->use_graphs = graphs != 0;
        if (cnn) c->gate_grid = grids[gi];
        skm_status s = skm_conceal_batch(c, frames, n, nullptr);   // warm (captures graphs)
        if (s != SKM_OK) return s;
        double t_best = 1e300;
        for (int r = 0; r < reps; ++r) {
          const auto t0 = std::chrono::steady_clock::now();
          if ((s = skm_conceal_batch(c, frames, n, nullptr)) != SKM_OK) return s;
          const double ms = std::chrono::duration<double, std::milli>(
                                std::chrono::steady_clock::now() - t0).count();
          if (ms < t_best) t_best = ms;
        }
        if (t_best < best) {
          best = t_best;
          bs = streams[si]; bg = graphs; bgg = c->gate_grid;
        }
      }
    }
  }
  c->batch_streams = bs;
  c->use_graphs = bg != 0;
  c->gate_grid = bgg;
  if (best_ms) *best_ms = best;
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
