// Host-callable launchers for one storage type S (explicitly instantiated in
// step_<type>.hip) plus the auxiliary per-node kernels: initialisation at the guided
// equilibrium, population export/import, moments, FP64 invariants, and the adjoint's
// seed and initial-condition kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace lbm {

// Everything a launcher needs to know about a run (host side).
// Every buffer is row-interleaved and lane-strided within a row: element (i, x, y) at
// y * row_stride + i * pitch + pos(x), pos(x) = (x mod S) * 64 + floor(x / S), S = pitch / 64.
struct RunDesc {
  int nx, ny, pitch;  // pitch = 64 ceil(nx / 64)
  int64_t rs;         // row stride of the populations and of fbar (9 * pitch)
  int64_t rs_rec;     // row stride of a recorded-moment slot (5 * pitch)
  double theta, nu, rho0, tau;
  int model;         // M_BGK ... M_COMPLETE
  int fuse_rb;       // row blocks of the two-step kernel; 0: one step per launch
  int adj_rb;        // row blocks of the two-step adjoint kernel; 0: one reverse step per launch
  int walls;         // 1: solid bounce-back columns at x = 0 and x = nx - 1 (A-B only)
  int wt_stores;     // 1: the step kernels' stores carry the SC1 scope bit (population buffers
                     // larger than the last-level cache; see kAuxStore)
};

// Population-buffer size from which the step kernels' stores are written through (SC1): the
// read and the written buffer of an A-B step then no longer fit the 256 MB last-level cache.
constexpr int64_t kWriteThroughBytes = int64_t(128) << 20;

// State layout at a given time: f_i(x) = buf[swap ? opp(i) : i][x - shift c_i].
struct LayoutSel {
  int shift, swap;
};

constexpr int kReduceBlocks = 1024;  // partial sums of the FP64 invariants

template <class S>
struct Engine {
  using T = typename StorageTraits<S>::T;
  static hipError_t step(const RunDesc& d, int phase, const void* src, void* dst, void* rec, hipStream_t st);
  // Two A-B steps in one launch (src and dst distinct) over d.fuse_rb row blocks, recording
  // both steps' moments to rec1/rec2 when they are not null. fuse_row_blocks gives the row
  // blocks for the current device (mode 0: only where it pays, 1: wherever the layout and
  // the storage type allow it), or 0 for one step per launch.
  static int fuse_row_blocks(const RunDesc& d, int mode);
  static int adjoint_row_blocks(const RunDesc& d, int mode);
  static hipError_t step2(const RunDesc& d, const void* src, void* dst, void* rec1, void* rec2, hipStream_t st);
  static hipError_t init(const RunDesc& d, LayoutSel L, void* buf, const double* rho, const double* ux,
                         const double* uy, hipStream_t st);
  static hipError_t get(const RunDesc& d, LayoutSel L, const void* buf, bool out_f64, void* out, hipStream_t st);
  static hipError_t set(const RunDesc& d, LayoutSel L, void* buf, const double* in, hipStream_t st);
  static hipError_t moments(const RunDesc& d, LayoutSel L, const void* buf, bool out_f64, void* rho, void* ux,
                            void* uy, hipStream_t st);
  static hipError_t invariants(const RunDesc& d, LayoutSel L, const void* buf, double* partial, double* result,
                               hipStream_t st);
  static hipError_t seed(const RunDesc& d, LayoutSel L, const void* buf, const T* rhob, const T* uxb,
                         const T* uyb, T* fbar, hipStream_t st);
  static hipError_t fbar_import(const RunDesc& d, const T* dense, T* fbar, hipStream_t st);
  static hipError_t fbar_export(const RunDesc& d, const T* fbar, T* dense, hipStream_t st);
  static hipError_t adjoint_step(const RunDesc& d, const T* fbar_next, T* fbar, const T* rec, hipStream_t st);
  // Two reverse steps (fbar^{n+1} -> fbar^{n-1}) over d.adj_rb row blocks; rec_hi holds the
  // records of step n, rec_lo those of step n - 1.
  static hipError_t adjoint_step2(const RunDesc& d, const T* fbar_next, T* fbar, const T* rec_hi, const T* rec_lo,
                                  hipStream_t st);
  static hipError_t ic_adjoint(const RunDesc& d, LayoutSel L, const void* buf0, const T* fbar, T* uxb, T* uyb,
                               hipStream_t st);
};

// Host-side construction of the per-run constants (FP64, rounded once to T).
template <class T>
inline Coef<T> make_coef(const RunDesc& d) {
  Coef<T> k;
  const double th = d.theta;
  k.rho0 = T(d.rho0);
  k.omb = T(1.0 - 1.0 / d.tau);
  k.omb_inv2th2 = T((1.0 - 1.0 / d.tau) / (2.0 * th * th));
  // Per-axis rest factors with r0 + 2 r1 == 1 exactly in T. The product equilibrium carries
  // momentum rho u (r0 + 2 r1) and density excess drho (r0 + 2 r1)^2, so a rounding excess
  // e = r0 + 2 r1 - 1 would scale the momentum field by 1 + e every step (1 + e/tau for LBGK):
  // with FP32 at theta = 1/3, e = 3e-8 and the kinetic energy gains 6e-5 per 1000 steps. The
  // difference that forms the second factor is exact (Sterbenz): 1 - r0 for r0 >= 1/2, and
  // 1 - 2 r1 for 2 r1 >= 1/2.
  if (th <= 0.5) {
    k.r0 = T(1.0 - th);
    k.r1 = (T(1) - k.r0) * T(0.5);
  } else {
    k.r1 = T(0.5 * th);
    k.r0 = T(1) - T(2) * k.r1;
  }
  k.rr0 = T(d.rho0 * double(k.r0));
  k.rr1 = T(d.rho0 * double(k.r1));
  k.inv2th2 = T(1.0 / (2.0 * th * th));
  k.inv4th2 = T(1.0 / (4.0 * th * th));
  k.inv8th2 = T(1.0 / (8.0 * th * th));
  k.a0 = T(th * (1.0 - 3.0 * th));
  k.b0 = T(2.0 * th * (1.0 - th));
  k.c3 = T(1.0 - 3.0 * th);
  return k;
}

}  // namespace lbm
