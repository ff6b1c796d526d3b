// Host runtime of liblbm.so: parameter validation, workspace planning, the time-step
// driver with sqrt(N) checkpointing, the adjoint sweep, and the C ABI declared in lbm.h.
// Device memory is never allocated here: every buffer lives in the caller's workspace.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <string>

#include "lbm_engine.h"

namespace lbm {
extern template struct Engine<double>;
extern template struct Engine<float>;
extern template struct Engine<_Float16>;
extern template struct Engine<bf16_t>;
}  // namespace lbm

namespace {

thread_local std::string g_last_error;

lbm_status fail(lbm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t storage_size(int dt) { return dt == LBM_F64 ? 8 : dt == LBM_F32 ? 4 : 2; }
size_t compute_size(int dt) { return dt == LBM_F64 ? 8 : 4; }

// Workspace regions (byte offsets into the caller's buffer).
struct Plan {
  size_t esize = 0, tsize = 0;        // storage / compute element sizes
  size_t pop_bytes = 0;               // one population set (storage type)
  size_t pop_off[2] = {0, 0};
  size_t red_off = 0, res_off = 0;
  int64_t stride = 0;                 // checkpoint spacing s
  int64_t nck = 0;                    // checkpoints at t = 0, s, 2s, ... (< N)
  size_t ckpt_off = 0;                // nck + 1 slots (the last holds the state at t = N)
  size_t rec_off = 0, rec_slot_bytes = 0;
  size_t fbar_off[2] = {0, 0}, fbar_bytes = 0;
  size_t total = 0;
};

// Elements per population row: nx rounded up to whole 64-node groups (lane-strided rows).
int64_t row_pitch(int64_t nx) { return (nx + 63) / 64 * 64; }

// Largest byte offset within one lattice row (its nine population rows, in the storage type
// or, for the adjoint's buffers, the compute type) that the kernels address: they add 32-bit
// in-row byte offsets to a row's base.
constexpr int64_t kMaxRowBytes = int64_t(1) << 31;

lbm_status validate(const lbm_params* p) {
  if (!p) return fail(LBM_ERR_INVALID_ARGUMENT, "params is NULL");
  if (p->nx < 1 || p->ny < 1) return fail(LBM_ERR_INVALID_ARGUMENT, "nx and ny must be >= 1");
  if (p->storage < LBM_F64 || p->storage > LBM_F16) return fail(LBM_ERR_INVALID_ARGUMENT, "unknown storage type");
  if (row_pitch(p->nx) * int64_t(p->ny) >= (int64_t(1) << 31))
    return fail(LBM_ERR_INVALID_ARGUMENT, "grid too large: (nx rounded up to 64) * ny must be < 2^31");
  const int64_t elem = int64_t(std::max(storage_size(p->storage), compute_size(p->storage)));
  if (int64_t(lbm::Q) * row_pitch(p->nx) * elem >= kMaxRowBytes)
    return fail(LBM_ERR_INVALID_ARGUMENT,
                "grid too wide: 9 * (nx rounded up to 64) * (larger of the storage and compute element sizes) "
                "must be < 2^31 bytes");
  if (!(p->theta > 0.0 && p->theta < 1.0)) return fail(LBM_ERR_INVALID_ARGUMENT, "theta must lie in (0, 1)");
  if (!(p->nu > 0.0) || !std::isfinite(p->nu)) return fail(LBM_ERR_INVALID_ARGUMENT, "nu must be finite and > 0");
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail(LBM_ERR_INVALID_ARGUMENT, "rho0 must be finite and > 0");
  if (p->model < LBM_BGK || p->model > LBM_OREG_COMPLETE) return fail(LBM_ERR_INVALID_ARGUMENT, "unknown model");
  if (p->pattern != LBM_AB && p->pattern != LBM_AA) return fail(LBM_ERR_INVALID_ARGUMENT, "unknown pattern");
  if (p->record_steps < 0) return fail(LBM_ERR_INVALID_ARGUMENT, "record_steps must be >= 0");
  if (p->ckpt_stride < 0) return fail(LBM_ERR_INVALID_ARGUMENT, "ckpt_stride must be >= 0");
  if (p->two_step < -1 || p->two_step > 1) return fail(LBM_ERR_INVALID_ARGUMENT, "two_step must be -1, 0 or 1");
  if (p->walls != 0 && p->walls != 1) return fail(LBM_ERR_INVALID_ARGUMENT, "walls must be 0 or 1");
  if (p->walls) {
    if (p->nx < 3) return fail(LBM_ERR_INVALID_ARGUMENT, "walls need nx >= 3");
    if (p->pattern != LBM_AB) return fail(LBM_ERR_UNSUPPORTED, "walls are implemented for the A-B pattern only");
    if (p->record_steps > 0) return fail(LBM_ERR_UNSUPPORTED, "walls are not implemented for recorded (adjoint) runs");
  }
  return LBM_OK;
}

Plan make_plan(const lbm_params& p) {
  Plan pl;
  pl.esize = storage_size(p.storage);
  pl.tsize = compute_size(p.storage);
  const size_t pitch = size_t(row_pitch(p.nx));
  // Row-interleaved buffers: ny rows of nine (populations) or five (recorded moments)
  // population rows of `pitch` elements each, rounded up to 4 KiB.
  pl.pop_bytes = round_up(size_t(lbm::Q) * pitch * p.ny * pl.esize, 4096);
  size_t off = 0;
  pl.pop_off[0] = off;
  off += pl.pop_bytes;
  if (p.pattern == LBM_AB) {
    pl.pop_off[1] = off;
    off += pl.pop_bytes;
  }
  pl.red_off = off;
  off += round_up(lbm::kReduceBlocks * 4 * sizeof(double), 256);
  pl.res_off = off;
  off += 256;
  if (p.record_steps > 0) {
    const int64_t N = p.record_steps;
    pl.stride = p.ckpt_stride > 0 ? p.ckpt_stride : int64_t(std::ceil(std::sqrt(double(N))));
    pl.stride = std::max<int64_t>(1, std::min<int64_t>(pl.stride, N));
    pl.nck = (N + pl.stride - 1) / pl.stride;
    pl.ckpt_off = off;
    off += size_t(pl.nck + 1) * pl.pop_bytes;
    pl.rec_slot_bytes = round_up(size_t(lbm::NREC) * pitch * p.ny * pl.tsize, 4096);
    pl.rec_off = off;
    off += size_t(pl.stride) * pl.rec_slot_bytes;
    pl.fbar_bytes = round_up(size_t(lbm::Q) * pitch * p.ny * pl.tsize, 4096);
    pl.fbar_off[0] = off;
    off += pl.fbar_bytes;
    pl.fbar_off[1] = off;
    off += pl.fbar_bytes;
  }
  pl.total = off;
  return pl;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

// Launch-bound grids: lbm_step replays a HIP graph of kGraphSteps step launches (an even
// count, so the A-B buffer index and the AA phase parity return to their start values)
// instead of launching every step from the host. Measured on MI355X: host-side launches
// cost 3.3 us per step, graph replays 0.8 us; per-step time at 64^2 and 128^2 drops from
// 3.3-3.5 to 2.5-3.1 us (the GPU's own dispatch of dependent kernels remains), at 256^2 it
// no longer improves (FP64 got slower), so graphs are used up to 2^15 storage positions.
constexpr int kGraphSteps = 64;
constexpr int64_t kGraphMaxPositions = int64_t(1) << 15;

struct lbm_ctx {
  lbm_params p;
  lbm::RunDesc d;
  Plan plan;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t time = 0;
  int cur = 0;            // A-B: buffer holding the state
  bool rec_valid = false; // recorded run usable by the adjoint
  // The record slots hold the moments of the last segment's steps, written by the forward
  // run, so the reverse sweep need not recompute that segment.
  bool last_seg_recorded = false;
  // Step graphs, built on first use: [A-B buffer index or AA phase parity at the start].
  hipStream_t capture = nullptr;  // private stream, used only to record the graphs
  hipGraphExec_t graph[2] = {nullptr, nullptr};

  ~lbm_ctx() {
    for (hipGraphExec_t& g : graph)
      if (g) (void)hipGraphExecDestroy(g);
    if (capture) (void)hipStreamDestroy(capture);
  }

  // The state lives in population buffer cur (A-B) or 0 (AA) or, during a recorded run,
  // in the checkpoint slot state_slot: a step that ends at a checkpoint time writes its
  // output there instead of copying it afterwards, and the next step reads it from there.
  int64_t state_slot = -1;
  void* state() const {
    return state_slot >= 0 ? ckpt(state_slot) : ws + plan.pop_off[p.pattern == LBM_AB ? cur : 0];
  }
  lbm::LayoutSel layout(int64_t t) const {
    if (p.pattern == LBM_AB) return {1, 0};
    return (t & 1) ? lbm::LayoutSel{1, 1} : lbm::LayoutSel{0, 0};
  }
  void* ckpt(int64_t k) const { return ws + plan.ckpt_off + size_t(k) * plan.pop_bytes; }
  void* rec_slot(int64_t j) const { return ws + plan.rec_off + size_t(j) * plan.rec_slot_bytes; }
  void* fbar(int b) const { return ws + plan.fbar_off[b]; }
};

namespace {

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(LBM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class F>
int dispatch_int(int storage, F&& f) {
  switch (storage) {
    case LBM_F64: return f(lbm::Engine<double>{});
    case LBM_F32: return f(lbm::Engine<float>{});
    case LBM_F16: return f(lbm::Engine<_Float16>{});
    default: return f(lbm::Engine<lbm::bf16_t>{});
  }
}

template <class F>
lbm_status dispatch(int storage, F&& f) {
  switch (storage) {
    case LBM_F64: return f(lbm::Engine<double>{});
    case LBM_F32: return f(lbm::Engine<float>{});
    case LBM_F16: return f(lbm::Engine<_Float16>{});
    default: return f(lbm::Engine<lbm::bf16_t>{});
  }
}

lbm_status check_ctx(const lbm_ctx* c) {
  if (!c) return fail(LBM_ERR_INVALID_ARGUMENT, "context is NULL");
  return LBM_OK;
}

lbm_status step_from(lbm_ctx* c, const void* src, void* rec);
lbm_status reduce_totals(lbm_ctx* c, double* partial, double* result, double out[3]);

// One time step of the current pattern; rec != nullptr also writes the moment record. A
// state held in a checkpoint slot is stepped out of place into population buffer 0.
lbm_status do_step(lbm_ctx* c, void* rec) {
  if (c->state_slot >= 0) return step_from(c, c->state(), rec);
  return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
    using E = decltype(eng);
    hipError_t e;
    if (c->p.pattern == LBM_AB) {
      e = E::step(c->d, lbm::PH_AB, c->ws + c->plan.pop_off[c->cur], c->ws + c->plan.pop_off[1 - c->cur], rec,
                  c->stream);
      if (e == hipSuccess) c->cur ^= 1;
    } else {
      const int ph = (c->time & 1) ? lbm::PH_AA_ODD : lbm::PH_AA_EVEN;
      e = E::step(c->d, ph, c->ws + c->plan.pop_off[0], c->ws + c->plan.pop_off[0], rec, c->stream);
    }
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("step kernel launch: ") + hipGetErrorString(e));
    ++c->time;
    return LBM_OK;
  });
}

// Two A-B steps in one launch (the LDS-staged kernel) from src into population buffer dst,
// which then holds the state; rec1/rec2 (or null) receive both steps' moment records.
lbm_status do_step2(lbm_ctx* c, const void* src, int dst, void* rec1, void* rec2) {
  return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
    using E = decltype(eng);
    const hipError_t e = E::step2(c->d, src, c->ws + c->plan.pop_off[dst], rec1, rec2, c->stream);
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("two-step kernel launch: ") + hipGetErrorString(e));
    c->cur = dst;
    c->state_slot = -1;
    c->time += 2;
    return LBM_OK;
  });
}

// One step (npair = 1) or an A-B pair (npair = 2) from the current state into checkpoint
// slot k, which then holds the state. Out of place, so valid for both AA phases as well.
lbm_status step_into_ckpt(lbm_ctx* c, int npair, int64_t k) {
  return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
    using E = decltype(eng);
    hipError_t e;
    if (npair == 2) {
      e = E::step2(c->d, c->state(), c->ckpt(k), nullptr, nullptr, c->stream);
    } else {
      const int ph = c->p.pattern == LBM_AB ? lbm::PH_AB : ((c->time & 1) ? lbm::PH_AA_ODD : lbm::PH_AA_EVEN);
      e = E::step(c->d, ph, c->state(), c->ckpt(k), nullptr, c->stream);
    }
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("step kernel launch: ") + hipGetErrorString(e));
    c->state_slot = k;
    c->cur = 0;
    c->time += npair;
    return LBM_OK;
  });
}

bool is_small(const lbm_ctx* c) { return int64_t(c->d.pitch) * c->d.ny <= kGraphMaxPositions; }

bool fused_ok(const lbm_ctx* c) { return c->d.fuse_rb > 0; }

// The executable graph of kGraphSteps steps from the current buffer index (A-B) or phase
// parity (AA). It is recorded by running the ordinary step launches against the private
// capture stream, with the context's stream, time and buffer index saved and restored:
// recording executes nothing and leaves the state as it was.
lbm_status step_graph(lbm_ctx* c, hipGraphExec_t* out) {
  const int key = c->p.pattern == LBM_AB ? c->cur : int(c->time & 1);
  if (!c->graph[key]) {
    if (!c->capture) HIP_TRY(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
    const hipStream_t user = c->stream;
    const int64_t t0 = c->time;
    const int cur0 = c->cur;
    HIP_TRY(hipStreamBeginCapture(c->capture, hipStreamCaptureModeRelaxed));
    c->stream = c->capture;
    lbm_status s = LBM_OK;
    for (int k = 0; k < kGraphSteps && s == LBM_OK; ++k) s = do_step(c, nullptr);
    c->stream = user;
    c->time = t0;
    c->cur = cur0;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->capture, &g);
    if (s == LBM_OK && e != hipSuccess) s = fail(LBM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    if (s == LBM_OK) {
      const hipError_t ei = hipGraphInstantiate(&c->graph[key], g, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        c->graph[key] = nullptr;
        s = fail(LBM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
      }
    }
    if (g) (void)hipGraphDestroy(g);
    if (s != LBM_OK) return s;
  }
  *out = c->graph[key];
  return LBM_OK;
}

// One step whose input is another buffer (a checkpoint slot), written to population buffer
// 0, which then holds the state. Valid for A-B and out of place for both AA phases: every
// node writes all nine of its output locations.
lbm_status step_from(lbm_ctx* c, const void* src, void* rec) {
  return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
    using E = decltype(eng);
    const int ph = c->p.pattern == LBM_AB ? lbm::PH_AB : ((c->time & 1) ? lbm::PH_AA_ODD : lbm::PH_AA_EVEN);
    const hipError_t e = E::step(c->d, ph, src, c->ws + c->plan.pop_off[0], rec, c->stream);
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("step kernel launch: ") + hipGetErrorString(e));
    c->cur = 0;
    c->state_slot = -1;
    ++c->time;
    return LBM_OK;
  });
}

lbm_status restore(lbm_ctx* c, int64_t slot, int64_t t) {
  HIP_TRY(hipMemcpyAsync(c->ws + c->plan.pop_off[0], c->ckpt(slot), c->plan.pop_bytes, hipMemcpyDeviceToDevice, c->stream));
  c->cur = 0;
  c->state_slot = -1;
  c->time = t;
  return LBM_OK;
}

// Reverse sweep over the recorded run: on entry fbar(0) holds dJ/df^N; on exit fbar(*out_b)
// holds dJ/df^0. Segment k (steps [k s, min((k+1) s, N))) is recomputed from its checkpoint
// while recording moments (two steps per launch where the two-step kernel applies; the
// first launch reads the checkpoint slot directly, so no copy restores it), then traversed
// backwards with the adjoint kernel. The last segment's moments are usually still in the
// slots from the forward run, which recorded them; with a single segment (stride >= N)
// nothing is recomputed at all.
lbm_status sweep(lbm_ctx* c, int* out_b) {
  const int64_t N = c->p.record_steps, s = c->plan.stride;
  int b = 0;
  for (int64_t k = c->plan.nck - 1; k >= 0; --k) {
    const int64_t t0 = k * s, t1 = std::min(t0 + s, N);
    lbm_status st = LBM_OK;
    if (!(k == c->plan.nck - 1 && c->last_seg_recorded)) {
      // The slots are about to hold this segment's moments (cleared first, so that a sweep
      // that fails part-way never leaves the flag on overwritten slots).
      c->last_seg_recorded = false;
      c->time = t0;
      const bool fz = fused_ok(c);
      st = (fz && t1 - t0 >= 2) ? do_step2(c, c->ckpt(k), 0, c->rec_slot(0), c->rec_slot(1))
                                : step_from(c, c->ckpt(k), c->rec_slot(0));
      if (st != LBM_OK) return st;
      while (c->time < t1) {
        const int64_t j = c->time - t0;
        st = (fz && t1 - c->time >= 2) ? do_step2(c, c->state(), 1 - c->cur, c->rec_slot(j), c->rec_slot(j + 1))
                                       : do_step(c, c->rec_slot(j));
        if (st != LBM_OK) return st;
      }
    }
    // Reverse steps t = t1 - 1 .. t0, two per launch (t and t - 1) where the two-step adjoint
    // kernel applies.
    for (int64_t t = t1 - 1; t >= t0;) {
      const bool pair = c->d.adj_rb > 0 && t - 1 >= t0;
      st = dispatch(c->p.storage, [&](auto eng) -> lbm_status {
        using E = decltype(eng);
        using T = typename E::T;
        const T* in = static_cast<const T*>(c->fbar(b));
        T* out = static_cast<T*>(c->fbar(1 - b));
        hipError_t e = pair ? E::adjoint_step2(c->d, in, out, static_cast<const T*>(c->rec_slot(t - t0)),
                                               static_cast<const T*>(c->rec_slot(t - 1 - t0)), c->stream)
                            : E::adjoint_step(c->d, in, out, static_cast<const T*>(c->rec_slot(t - t0)), c->stream);
        if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("adjoint kernel launch: ") + hipGetErrorString(e));
        return LBM_OK;
      });
      if (st != LBM_OK) return st;
      b ^= 1;
      t -= pair ? 2 : 1;
    }
  }
  *out_b = b;
  return LBM_OK;
}

// True when the reverse sweep will recompute nothing (one segment, its moments kept by the
// forward run): the state at N is then never touched and needs no saving and restoring.
bool state_stays(const lbm_ctx* c) { return c->plan.nck == 1 && c->last_seg_recorded; }

lbm_status check_adjoint_ready(const lbm_ctx* c) {
  if (c->p.record_steps <= 0) return fail(LBM_ERR_STATE, "context was created with record_steps = 0");
  if (!c->rec_valid) return fail(LBM_ERR_STATE, "recorded run was invalidated by lbm_set_populations");
  if (c->time != c->p.record_steps)
    return fail(LBM_ERR_STATE, "lbm_time must equal record_steps (" + std::to_string(c->p.record_steps) + "), is " +
                                   std::to_string(c->time));
  return LBM_OK;
}

template <class F>
lbm_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(LBM_ERR_INVALID_ARGUMENT, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(LBM_ERR_INVALID_ARGUMENT, e.what());
  } catch (...) {
    return fail(LBM_ERR_INVALID_ARGUMENT, "unknown exception");
  }
}

}  // namespace

extern "C" {

lbm_status lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
  return guarded([&]() -> lbm_status {
    lbm_status s = validate(p);
    if (s != LBM_OK) return s;
    if (!bytes) return fail(LBM_ERR_INVALID_ARGUMENT, "bytes is NULL");
    *bytes = make_plan(*p).total;
    return LBM_OK;
  });
}

lbm_status lbm_init(const lbm_params* p, void* d_workspace, size_t workspace_bytes, void* hip_stream,
                    const double* d_rho, const double* d_ux, const double* d_uy, lbm_ctx** out) {
  return guarded([&]() -> lbm_status {
    if (!out) return fail(LBM_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    lbm_status s = validate(p);
    if (s != LBM_OK) return s;
    if (!d_workspace) return fail(LBM_ERR_INVALID_ARGUMENT, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
      return fail(LBM_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    if (!d_ux || !d_uy) return fail(LBM_ERR_INVALID_ARGUMENT, "velocity fields are required");
    const Plan plan = make_plan(*p);
    if (workspace_bytes < plan.total)
      return fail(LBM_ERR_WORKSPACE_TOO_SMALL, "workspace has " + std::to_string(workspace_bytes) + " bytes, needs " +
                                                   std::to_string(plan.total));
    lbm_ctx* c = new lbm_ctx();
    c->p = *p;
    c->plan = plan;
    c->ws = static_cast<char*>(d_workspace);
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
    lbm::RunDesc& d = c->d;
    d.nx = p->nx;
    d.ny = p->ny;
    d.pitch = int(row_pitch(p->nx));
    d.rs = int64_t(lbm::Q) * d.pitch;
    d.rs_rec = int64_t(lbm::NREC) * d.pitch;
    d.theta = p->theta;
    d.nu = p->nu;
    d.rho0 = p->rho0;
    d.tau = p->nu / p->theta + 0.5;  // nu = theta (tau - 1/2)
    d.model = p->model;
    d.walls = p->walls;
    d.wt_stores = int64_t(lbm::Q) * d.pitch * d.ny * int64_t(storage_size(p->storage)) >= lbm::kWriteThroughBytes;
    d.fuse_rb = (p->pattern == LBM_AB && p->two_step >= 0 && !p->walls)
                    ? dispatch_int(p->storage, [&](auto eng) { return decltype(eng)::fuse_row_blocks(d, p->two_step); })
                    : 0;
    d.adj_rb = (p->record_steps > 0 && p->two_step >= 0)
                   ? dispatch_int(p->storage, [&](auto eng) { return decltype(eng)::adjoint_row_blocks(d, p->two_step); })
                   : 0;
    c->time = 0;
    c->cur = 0;
    c->rec_valid = p->record_steps > 0;
    c->state_slot = c->rec_valid ? 0 : -1;  // a recorded run's initial state is checkpoint 0
    s = dispatch(p->storage, [&](auto eng) -> lbm_status {
      using E = decltype(eng);
      hipError_t e = E::init(c->d, c->layout(0), c->state(), d_rho, d_ux, d_uy, c->stream);
      if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("init kernel launch: ") + hipGetErrorString(e));
      return LBM_OK;
    });
    if (s != LBM_OK) {
      delete c;
      return s;
    }
    *out = c;
    return LBM_OK;
  });
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  return guarded([&]() -> lbm_status {
    lbm_status s = check_ctx(c);
    if (s != LBM_OK) return s;
    if (n < 0) return fail(LBM_ERR_INVALID_ARGUMENT, "n must be >= 0");
    DeviceGuard g(c->device);
    const int64_t N = c->p.record_steps;
    const bool small = is_small(c);
    const bool fused = !small && fused_ok(c);
    const int64_t t_last = N > 0 ? (c->plan.nck - 1) * c->plan.stride : 0;  // last segment's start
    for (int64_t k = 0; k < n;) {
      const bool recording = N > 0 && c->rec_valid && c->time < N;
      // The checkpoint of a checkpoint time: normally the step that ended here wrote the
      // state into its slot; otherwise (a state replaced at t = 0) it is copied.
      if (recording && c->time % c->plan.stride == 0 && c->state_slot != c->time / c->plan.stride)
        HIP_TRY(hipMemcpyAsync(c->ckpt(c->time / c->plan.stride), c->state(), c->plan.pop_bytes,
                               hipMemcpyDeviceToDevice, c->stream));
      // Steps of the last segment keep their moments for the reverse sweep (slot t - t_last).
      const bool keep = recording && c->time >= t_last;
      // A pair of steps must not pass over a checkpoint time of the recorded window, nor
      // over its end while keeping moments.
      const int64_t mid = c->time + 1;
      const bool pair =
          fused && n - k >= 2 && !(recording && mid < N && mid % c->plan.stride == 0) && !(keep && mid >= N);
      // A step that ends at a later checkpoint time of the window writes into its slot (never
      // while keeping moments: the last segment holds no further checkpoint time).
      const int64_t end = c->time + (pair ? 2 : 1);
      const bool into_ckpt = recording && end < N && end % c->plan.stride == 0;
      if (into_ckpt) {
        s = step_into_ckpt(c, pair ? 2 : 1, end / c->plan.stride);
        if (s != LBM_OK) return s;
        k += pair ? 2 : 1;
        continue;
      }
      if (pair) {
        const int64_t j = c->time - t_last;
        s = keep ? do_step2(c, c->state(), 1 - c->cur, c->rec_slot(j), c->rec_slot(j + 1))
                 : do_step2(c, c->state(), 1 - c->cur, nullptr, nullptr);
        if (s != LBM_OK) return s;
        if (keep && c->time == N) c->last_seg_recorded = true;
        k += 2;
        continue;
      }
      if (small && !recording && c->state_slot < 0 && n - k >= kGraphSteps) {
        hipGraphExec_t ge = nullptr;
        s = step_graph(c, &ge);
        if (s != LBM_OK) return s;
        HIP_TRY(hipGraphLaunch(ge, c->stream));
        c->time += kGraphSteps;  // even count: buffer index and phase parity unchanged
        k += kGraphSteps;
        continue;
      }
      s = do_step(c, keep ? c->rec_slot(c->time - t_last) : nullptr);
      if (s != LBM_OK) return s;
      if (keep && c->time == N) c->last_seg_recorded = true;
      ++k;
    }
    return LBM_OK;
  });
}

lbm_status lbm_moments(lbm_ctx* c, lbm_dtype out_dtype, void* d_rho, void* d_ux, void* d_uy) {
  return guarded([&]() -> lbm_status {
    lbm_status s = check_ctx(c);
    if (s != LBM_OK) return s;
    if (out_dtype != LBM_F64 && out_dtype != LBM_F32) return fail(LBM_ERR_UNSUPPORTED, "moments: output must be F64 or F32");
    DeviceGuard g(c->device);
    return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
      using E = decltype(eng);
      hipError_t e = E::moments(c->d, c->layout(c->time), c->state(), out_dtype == LBM_F64, d_rho, d_ux, d_uy, c->stream);
      if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("moments kernel launch: ") + hipGetErrorString(e));
      return LBM_OK;
    });
  });
}

lbm_status lbm_get_populations(lbm_ctx* c, lbm_dtype out_dtype, void* d_f) {
  return guarded([&]() -> lbm_status {
    lbm_status s = check_ctx(c);
    if (s != LBM_OK) return s;
    if (!d_f) return fail(LBM_ERR_INVALID_ARGUMENT, "output is NULL");
    if (out_dtype != LBM_F64 && out_dtype != LBM_F32) return fail(LBM_ERR_UNSUPPORTED, "populations: output must be F64 or F32");
    DeviceGuard g(c->device);
    return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
      using E = decltype(eng);
      hipError_t e = E::get(c->d, c->layout(c->time), c->state(), out_dtype == LBM_F64, d_f, c->stream);
      if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("export kernel launch: ") + hipGetErrorString(e));
      return LBM_OK;
    });
  });
}

lbm_status lbm_set_populations(lbm_ctx* c, const double* d_f) {
  return guarded([&]() -> lbm_status {
    lbm_status s = check_ctx(c);
    if (s != LBM_OK) return s;
    if (!d_f) return fail(LBM_ERR_INVALID_ARGUMENT, "input is NULL");
    DeviceGuard g(c->device);
    if (c->time != 0) c->rec_valid = false;
    c->last_seg_recorded = false;
    // The new state goes to a population buffer; a checkpoint slot keeps what it holds.
    if (c->state_slot >= 0) {
      c->state_slot = -1;
      c->cur = 0;
    }
    return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
      using E = decltype(eng);
      hipError_t e = E::set(c->d, c->layout(c->time), c->state(), d_f, c->stream);
      if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("import kernel launch: ") + hipGetErrorString(e));
      return LBM_OK;
    });
  });
}

lbm_status lbm_invariants(lbm_ctx* c, double out[3]) {
  return guarded([&]() -> lbm_status {
    lbm_status s = check_ctx(c);
    if (s != LBM_OK) return s;
    if (!out) return fail(LBM_ERR_INVALID_ARGUMENT, "out is NULL");
    DeviceGuard g(c->device);
    return reduce_totals(c, reinterpret_cast<double*>(c->ws + c->plan.red_off),
                         reinterpret_cast<double*>(c->ws + c->plan.res_off), out);
  });
}

}  // extern "C"

namespace {

// Reduction scratch of lbm_invariants_static: kReduceBlocks x 4 FP64 partial sums followed by
// the 4-entry result (sum rho, sum rho u_x, sum rho u_y, non-finite count). Every device the
// library runs on holds its own copy until the process ends. In host code `scratch` names a
// host-side stand-in, not device memory: kernels and copies use the address that
// hipGetSymbolAddress returns for the current device, kept per device below.
constexpr size_t kStaticScratchDoubles = size_t(lbm::kReduceBlocks) * 4 + 4;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;

// Device address of `dev`'s copy of the scratch array, looked up once per device with that
// device current (the caller makes it current).
lbm_status static_scratch(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    double* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LBM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return LBM_OK;
}

// The two reduction kernels of the FP64 totals with their partials and result at `partial`
// and `result`, then the result copied to the host after the stream has drained.
lbm_status reduce_totals(lbm_ctx* c, double* partial, double* result, double out[3]) {
  lbm_status s = dispatch(c->p.storage, [&](auto eng) -> lbm_status {
    using E = decltype(eng);
    hipError_t e = E::invariants(c->d, c->layout(c->time), c->state(), partial, result, c->stream);
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("reduction kernel launch: ") + hipGetErrorString(e));
    return LBM_OK;
  });
  if (s != LBM_OK) return s;
  double host[4];
  HIP_TRY(hipMemcpyAsync(host, result, sizeof(host), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  out[0] = host[0];
  out[1] = host[1];
  out[2] = host[2];
  if (host[3] > 0.0) return fail(LBM_ERR_NONFINITE, std::to_string(int64_t(host[3])) + " nodes hold non-finite populations");
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_invariants_static(lbm_ctx* c, double out[3]) {
  return guarded([&]() -> lbm_status {
    lbm_status s = check_ctx(c);
    if (s != LBM_OK) return s;
    if (!out) return fail(LBM_ERR_INVALID_ARGUMENT, "out is NULL");
    DeviceGuard g(c->device);
    double* ptr = nullptr;
    s = static_scratch(c->device, &ptr);
    if (s != LBM_OK) return s;
    // The partial count is fixed (it does not grow with the grid), so every grid lbm_init
    // accepts fits the array; the check guards the layout itself.
    if (size_t(lbm::kReduceBlocks) * 4 + 4 > kStaticScratchDoubles)
      return fail(LBM_ERR_UNSUPPORTED, "reduction partials exceed the static scratch array");
    // Every partial and the result are written by the kernels before they are read, so the
    // array needs no clearing between calls.
    return reduce_totals(c, ptr, ptr + size_t(lbm::kReduceBlocks) * 4, out);
  });
}

lbm_status lbm_adjoint(lbm_ctx* c, const void* d_rho_bar, const void* d_ux_bar, const void* d_uy_bar,
                       void* d_ux0_bar, void* d_uy0_bar) {
  return guarded([&]() -> lbm_status {
    lbm_status s = check_ctx(c);
    if (s != LBM_OK) return s;
    s = check_adjoint_ready(c);
    if (s != LBM_OK) return s;
    if (!d_ux_bar || !d_uy_bar || !d_ux0_bar || !d_uy0_bar)
      return fail(LBM_ERR_INVALID_ARGUMENT, "adjoint: velocity adjoint pointers are required");
    DeviceGuard g(c->device);
    const int64_t N = c->p.record_steps;
    const bool in_place = state_stays(c);
    if (!in_place)
      HIP_TRY(hipMemcpyAsync(c->ckpt(c->plan.nck), c->state(), c->plan.pop_bytes, hipMemcpyDeviceToDevice, c->stream));
    return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
      using E = decltype(eng);
      using T = typename E::T;
      hipError_t e = E::seed(c->d, c->layout(N), c->state(), static_cast<const T*>(d_rho_bar),
                             static_cast<const T*>(d_ux_bar), static_cast<const T*>(d_uy_bar),
                             static_cast<T*>(c->fbar(0)), c->stream);
      if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("seed kernel launch: ") + hipGetErrorString(e));
      int b = 0;
      lbm_status st = sweep(c, &b);
      if (st != LBM_OK) return st;
      e = E::ic_adjoint(c->d, c->layout(0), c->ckpt(0), static_cast<const T*>(c->fbar(b)), static_cast<T*>(d_ux0_bar),
                        static_cast<T*>(d_uy0_bar), c->stream);
      if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("initial-condition adjoint launch: ") + hipGetErrorString(e));
      return in_place ? LBM_OK : restore(c, c->plan.nck, N);
    });
  });
}

lbm_status lbm_adjoint_populations(lbm_ctx* c, const void* d_fbarN, void* d_fbar0) {
  return guarded([&]() -> lbm_status {
    lbm_status s = check_ctx(c);
    if (s != LBM_OK) return s;
    s = check_adjoint_ready(c);
    if (s != LBM_OK) return s;
    if (!d_fbarN || !d_fbar0) return fail(LBM_ERR_INVALID_ARGUMENT, "adjoint: population pointers are required");
    DeviceGuard g(c->device);
    const int64_t N = c->p.record_steps;
    const bool in_place = state_stays(c);
    if (!in_place)
      HIP_TRY(hipMemcpyAsync(c->ckpt(c->plan.nck), c->state(), c->plan.pop_bytes, hipMemcpyDeviceToDevice, c->stream));
    return dispatch(c->p.storage, [&](auto eng) -> lbm_status {
      using E = decltype(eng);
      using T = typename E::T;
      hipError_t e = E::fbar_import(c->d, static_cast<const T*>(d_fbarN), static_cast<T*>(c->fbar(0)), c->stream);
      if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("adjoint import launch: ") + hipGetErrorString(e));
      int b = 0;
      lbm_status st = sweep(c, &b);
      if (st != LBM_OK) return st;
      e = E::fbar_export(c->d, static_cast<const T*>(c->fbar(b)), static_cast<T*>(d_fbar0), c->stream);
      if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("adjoint export launch: ") + hipGetErrorString(e));
      return in_place ? LBM_OK : restore(c, c->plan.nck, N);
    });
  });
}

int32_t lbm_steps_per_launch(const lbm_ctx* c) {
  if (!c) return -1;
  return (!is_small(c) && fused_ok(c)) ? 2 : 1;
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->time : -1; }

const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "LBM_OK";
    case LBM_ERR_INVALID_ARGUMENT: return "LBM_ERR_INVALID_ARGUMENT";
    case LBM_ERR_UNSUPPORTED: return "LBM_ERR_UNSUPPORTED";
    case LBM_ERR_WORKSPACE_TOO_SMALL: return "LBM_ERR_WORKSPACE_TOO_SMALL";
    case LBM_ERR_HIP: return "LBM_ERR_HIP";
    case LBM_ERR_NONFINITE: return "LBM_ERR_NONFINITE";
    case LBM_ERR_STATE: return "LBM_ERR_STATE";
  }
  return "LBM_ERR_UNKNOWN";
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  delete c;
}

}  // extern "C"
