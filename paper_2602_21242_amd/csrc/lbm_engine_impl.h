// Definitions of Engine<S> (see lbm_engine.h). Included once per storage type.
#pragma once

#include <algorithm>

#include "lbm_engine.h"
#include "lbm_step.h"

namespace lbm {

// --- geometry -----------------------------------------------------------------------------

__host__ __device__ __forceinline__ int row_pos(int x, int S) { return (x % S) * kLanes + x / S; }

inline Geo make_geo(const RunDesc& d, int npt) {
  Geo g;
  g.nx = d.nx;
  g.ny = d.ny;
  g.S = d.pitch / kLanes;
  g.ps = d.pitch;
  g.rs = d.rs;
  const int groups_per_block = (kBlock / kLanes) * npt;
  g.nseg = (g.S + groups_per_block - 1) / groups_per_block;
  g.plast = row_pos(d.nx - 1, g.S);
  return g;
}

inline dim3 step_grid(const Geo& g) {
  return dim3(unsigned(g.nseg), unsigned(std::min(g.ny, kRowsY)), unsigned((g.ny + kRowsY - 1) / kRowsY));
}

// The auxiliary kernels run one thread per storage position (pitch * ny of them), so their
// nine population accesses are coalesced; the dense [ny][nx] fields are indexed by node.
inline int node_blocks(const RunDesc& d) { return int((int64_t(d.pitch) * d.ny + kBlock - 1) / kBlock); }

// Storage position t (row y, in-row position q) -> node x; false for padding and past the end.
__device__ __forceinline__ bool storage_node(int64_t t, const RunDesc& d, int& y, int& q, int& x) {
  if (t >= int64_t(d.pitch) * d.ny) return false;
  y = int(t / d.pitch);
  q = int(t - int64_t(y) * d.pitch);
  x = (q % kLanes) * (d.pitch / kLanes) + q / kLanes;
  return x < d.nx;
}

// Buffer index of population i of node (x, y) under a stored-state convention L.
__device__ __forceinline__ int64_t layout_index(int i, int x, int y, const RunDesc& d, LayoutSel L) {
  const int slot = L.swap ? opp(i) : i;
  int xs = x - L.shift * cx(i);
  xs = xs < 0 ? xs + d.nx : (xs >= d.nx ? xs - d.nx : xs);
  int ys = y - L.shift * cy(i);
  ys = ys < 0 ? ys + d.ny : (ys >= d.ny ? ys - d.ny : ys);
  return int64_t(ys) * d.rs + slot * d.pitch + row_pos(xs, d.pitch / kLanes);
}

// Buffer index of entry i of node (x, y) stored at in-row position q (no shift).
__device__ __forceinline__ int64_t local_index(int i, int q, int y, const RunDesc& d) {
  return int64_t(y) * d.rs + i * d.pitch + q;
}

// --- per-node auxiliary kernels --------------------------------------------------------------

// The per-node auxiliary kernels exchange the dense [ny][nx] fields through LDS: a
// block takes kTileGroups groups of one row (one wavefront per group, lane l holding node
// x = l S + s as in the storage layout), and the dense entries of those nodes -- kTileGroups
// consecutive x per lane -- are read or written by consecutive threads. (Indexing the dense
// fields by each thread's own node strides a wavefront's accesses by S elements.)
constexpr int kTileGroups = kBlock / kLanes;
inline dim3 tile_grid(const RunDesc& d) {
  const int S = d.pitch / kLanes;
  return dim3(unsigned((S + kTileGroups - 1) / kTileGroups), unsigned(std::min(d.ny, kRowsY)),
              unsigned((d.ny + kRowsY - 1) / kRowsY));
}
// A block's row y, its first group s0 and the group count S; for the thread's dense entry
// the lane lt, the group offset jt and the node x (-1 outside the row or in the padding).
struct Tile {
  int y, s0, S, lt, jt, xt;
};
__device__ __forceinline__ Tile tile_of(const RunDesc& d) {
  Tile t;
  t.y = int(blockIdx.z) * kRowsY + int(blockIdx.y);
  t.S = d.pitch / kLanes;
  t.s0 = int(blockIdx.x) * kTileGroups;
  t.lt = int(threadIdx.x) / kTileGroups;
  t.jt = int(threadIdx.x) % kTileGroups;
  const int x = t.lt * t.S + t.s0 + t.jt;
  t.xt = (t.s0 + t.jt < t.S && x < d.nx) ? x : -1;
  return t;
}


// f^0 = f^eq(rho, u) of the guided equilibrium (eq:guidedEq), stored shifted, computed from
// the caller's FP64 fields in FP64 as drho Phi_x Phi_y + rho0 (d_x Phi_y + r_x d_y) (no
// cancellation against w_i rho0) and rounded once to the storage type.
template <class S>
__global__ void __launch_bounds__(kBlock)
k_init(S* buf, RunDesc d, LayoutSel L, const double* rho, const double* ux, const double* uy) {
  using Tr = StorageTraits<S>;
  __shared__ double sh[3][kTileGroups][kLanes];
  const Tile tl = tile_of(d);
  if (tl.y >= d.ny) return;  // whole block
  if (tl.xt >= 0) {
    const int64_t n = int64_t(tl.y) * d.nx + tl.xt;
    sh[0][tl.jt][tl.lt] = rho ? rho[n] : d.rho0;
    sh[1][tl.jt][tl.lt] = ux[n];
    sh[2][tl.jt][tl.lt] = uy[n];
  }
  __syncthreads();
  const int w = int(threadIdx.x) / kLanes, lane = int(threadIdx.x) % kLanes;
  const int s = tl.s0 + w, x = lane * tl.S + s, y = tl.y;
  if (s >= tl.S || x >= d.nx) return;
  const double r = sh[0][w][lane];
  const double vx = sh[1][w][lane], vy = sh[2][w][lane];
  const double drho = r - d.rho0;
  const double th = d.theta;
  const double dx[3] = {0.5 * (vx * vx - vx), -vx * vx, 0.5 * (vx * vx + vx)};
  const double dy[3] = {0.5 * (vy * vy - vy), -vy * vy, 0.5 * (vy * vy + vy)};
  const double rr[3] = {0.5 * th, 1.0 - th, 0.5 * th};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int a = cx(i) + 1, b = cy(i) + 1;
    const double hx = rr[a] + dx[a], hy = rr[b] + dy[b];
    const double feqs = drho * hx * hy + d.rho0 * (dx[a] * hy + rr[a] * dy[b]);
    buf[layout_index(i, x, y, d, L)] = Tr::from_f64(feqs);
  }
}

// Export to FP64 or FP32: f = g + w rho0 in FP64 (exact for every storage type's g before the
// addition), rounded once to the output type.
template <class S, class O>
__global__ void __launch_bounds__(kBlock)
k_get(const S* buf, RunDesc d, LayoutSel L, O* out) {
  using Tr = StorageTraits<S>;
  __shared__ O sh[Q][kTileGroups][kLanes];
  const int64_t N = int64_t(d.nx) * d.ny;
  const Tile tl = tile_of(d);
  if (tl.y >= d.ny) return;  // whole block
  const int w = int(threadIdx.x) / kLanes, lane = int(threadIdx.x) % kLanes;
  const int s = tl.s0 + w, x = lane * tl.S + s, y = tl.y;
  if (s < tl.S && x < d.nx) {
    const double th = d.theta;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double wt = (cx(i) == 0 ? 1.0 - th : 0.5 * th) * (cy(i) == 0 ? 1.0 - th : 0.5 * th);
      const double g = double(Tr::load(buf[layout_index(i, x, y, d, L)]));
      sh[i][w][lane] = O(g + wt * d.rho0);
    }
  }
  __syncthreads();
  if (tl.xt >= 0) {
    const int64_t n = int64_t(y) * d.nx + tl.xt;
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i * N + n] = sh[i][tl.jt][tl.lt];
  }
}

// Import of the caller's FP64 populations: g = f - w rho0 in FP64, rounded once to the
// storage type.
template <class S>
__global__ void __launch_bounds__(kBlock)
k_set(S* buf, RunDesc d, LayoutSel L, const double* in) {
  using Tr = StorageTraits<S>;
  __shared__ double sh[Q][kTileGroups][kLanes];
  const int64_t N = int64_t(d.nx) * d.ny;
  const Tile tl = tile_of(d);
  if (tl.y >= d.ny) return;  // whole block
  if (tl.xt >= 0) {
    const int64_t n = int64_t(tl.y) * d.nx + tl.xt;
#pragma unroll
    for (int i = 0; i < Q; ++i) sh[i][tl.jt][tl.lt] = in[i * N + n];
  }
  __syncthreads();
  const int w = int(threadIdx.x) / kLanes, lane = int(threadIdx.x) % kLanes;
  const int s = tl.s0 + w, x = lane * tl.S + s, y = tl.y;
  if (s >= tl.S || x >= d.nx) return;
  const double th = d.theta;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double wt = (cx(i) == 0 ? 1.0 - th : 0.5 * th) * (cy(i) == 0 ? 1.0 - th : 0.5 * th);
    buf[layout_index(i, x, y, d, L)] = Tr::from_f64(sh[i][w][lane] - wt * d.rho0);
  }
}

// rho - rho0 and j of one node from the stored state, accumulated in A: FP64 for the global
// totals, the compute type for everything else.
template <class A, class S>
__device__ __forceinline__ void node_moments(const S* buf, const RunDesc& d, LayoutSel L, int x, int y,
                                             A& drho, A& jx, A& jy, bool* bad = nullptr) {
  using Tr = StorageTraits<S>;
  drho = jx = jy = A(0);
  bool nf = false;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const A g = A(Tr::load(buf[layout_index(i, x, y, d, L)]));
    nf |= !isfinite(g);
    drho += g;
    jx += A(cx(i)) * g;
    jy += A(cy(i)) * g;
  }
  if (bad) *bad = nf;
}

// rho and u = j / rho of every node, in the compute type, written as O.
template <class S, class O>
__global__ void __launch_bounds__(kBlock)
k_moments(const S* buf, RunDesc d, LayoutSel L, O* rho, O* ux, O* uy) {
  using T = typename StorageTraits<S>::T;
  __shared__ O sh[3][kTileGroups][kLanes];
  const Tile tl = tile_of(d);
  if (tl.y >= d.ny) return;  // whole block
  const int w = int(threadIdx.x) / kLanes, lane = int(threadIdx.x) % kLanes;
  const int s = tl.s0 + w, x = lane * tl.S + s, y = tl.y;
  if (s < tl.S && x < d.nx) {
    T drho, jx, jy;
    node_moments(buf, d, L, x, y, drho, jx, jy);
    const T r = T(d.rho0) + drho;
    sh[0][w][lane] = O(r);
    sh[1][w][lane] = O(jx / r);
    sh[2][w][lane] = O(jy / r);
  }
  __syncthreads();
  if (tl.xt >= 0) {
    const int64_t n = int64_t(y) * d.nx + tl.xt;
    if (rho) rho[n] = sh[0][tl.jt][tl.lt];
    if (ux) ux[n] = sh[1][tl.jt][tl.lt];
    if (uy) uy[n] = sh[2][tl.jt][tl.lt];
  }
}

// FP64 totals, first stage: fixed grid of kReduceBlocks blocks, deterministic order.
template <class S>
__global__ void __launch_bounds__(kBlock)
k_reduce_partial(const S* buf, RunDesc d, LayoutSel L, double* partial) {
  __shared__ double sh[4][kBlock];
  const int64_t T = int64_t(d.pitch) * d.ny;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x; t < T; t += int64_t(gridDim.x) * kBlock) {
    int y, q, x;
    if (!storage_node(t, d, y, q, x)) continue;
    double drho, jx, jy;
    bool bad;
    node_moments<double>(buf, d, L, x, y, drho, jx, jy, &bad);
    s0 += drho;
    s1 += jx;
    s2 += jy;
    s3 += bad ? 1.0 : 0.0;
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  sh[2][threadIdx.x] = s2;
  sh[3][threadIdx.x] = s3;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// Second stage: one block sums the partials; result = {sum rho, sum jx, sum jy, #non-finite}.
template <class S>
__global__ void __launch_bounds__(kBlock)
k_reduce_final(const double* partial, int nparts, double mass_offset, double* result) {
  __shared__ double sh[4][kBlock];
  double s[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += kBlock)
    for (int c = 0; c < 4; ++c) s[c] += partial[b * 4 + c];
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    result[0] = mass_offset + sh[0][0];
    result[1] = sh[1][0];
    result[2] = sh[2][0];
    result[3] = sh[3][0];
  }
}

// Adjoint seed: fbar^N_i = rho_bar + u_bar . (c_i - u)/rho (derivative of rho and
// u = sum c f / rho with respect to f_i), written to fbar (population layout, compute type).
// Seed of the reverse sweep: fbar^N_i = rho_bar + (u_bar . (c_i - u)) / rho, the adjoint of
// the moments (rho, u) at t = N with respect to the populations.
template <class S, class T>
__global__ void __launch_bounds__(kBlock)
k_seed(const S* buf, RunDesc d, LayoutSel L, const T* rhob, const T* uxb, const T* uyb, T* fbar) {
  __shared__ T sh[3][kTileGroups][kLanes];
  const Tile tl = tile_of(d);
  if (tl.y >= d.ny) return;  // whole block
  if (tl.xt >= 0) {
    const int64_t n = int64_t(tl.y) * d.nx + tl.xt;
    sh[0][tl.jt][tl.lt] = rhob ? rhob[n] : T(0);
    sh[1][tl.jt][tl.lt] = uxb[n];
    sh[2][tl.jt][tl.lt] = uyb[n];
  }
  __syncthreads();
  const int w = int(threadIdx.x) / kLanes, lane = int(threadIdx.x) % kLanes;
  const int s = tl.s0 + w, x = lane * tl.S + s, y = tl.y;
  if (s >= tl.S || x >= d.nx) return;
  const int q = s * kLanes + lane;
  T drho, jx, jy;
  node_moments(buf, d, L, x, y, drho, jx, jy);
  const T r = T(d.rho0) + drho;
  const T vx = jx / r, vy = jy / r;
  const T rb = sh[0][w][lane];
  const T ax = sh[1][w][lane] / r, ay = sh[2][w][lane] / r;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    fbar[local_index(i, q, y, d)] = rb + ax * (T(cx(i)) - vx) + ay * (T(cy(i)) - vy);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_fbar_import(RunDesc d, const T* dense, T* fbar) {
  const int64_t N = int64_t(d.nx) * d.ny;
  int y, q, x;
  if (!storage_node(int64_t(blockIdx.x) * kBlock + threadIdx.x, d, y, q, x)) return;
  const int64_t n = int64_t(y) * d.nx + x;
#pragma unroll
  for (int i = 0; i < Q; ++i) fbar[local_index(i, q, y, d)] = dense[i * N + n];
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_fbar_export(RunDesc d, const T* fbar, T* dense) {
  const int64_t N = int64_t(d.nx) * d.ny;
  int y, q, x;
  if (!storage_node(int64_t(blockIdx.x) * kBlock + threadIdx.x, d, y, q, x)) return;
  const int64_t n = int64_t(y) * d.nx + x;
#pragma unroll
  for (int i = 0; i < Q; ++i) dense[i * N + n] = fbar[local_index(i, q, y, d)];
}

// Initial-condition adjoint: f^0 = f^eq(rho0_field, u0) with rho held fixed, so
// u0bar_a = sum_i fbar^0_i d f_i^eq / d u_a, with dPhi(0,u)/du = -2u, dPhi(+-1,u)/du = u +- 1/2.
// rho and u are the moments of the recorded state at t = 0.
template <class S, class T>
__global__ void __launch_bounds__(kBlock)
k_ic_adjoint(const S* buf0, RunDesc d, LayoutSel L, const T* fbar, T* uxb, T* uyb) {
  __shared__ T sh[2][kTileGroups][kLanes];
  const Tile tl = tile_of(d);
  if (tl.y >= d.ny) return;  // whole block
  const int w = int(threadIdx.x) / kLanes, lane = int(threadIdx.x) % kLanes;
  const int s = tl.s0 + w, x = lane * tl.S + s, y = tl.y;
  if (s < tl.S && x < d.nx) {
    const int q = s * kLanes + lane;
    T drho, jx, jy;
    node_moments(buf0, d, L, x, y, drho, jx, jy);
    const T r = T(d.rho0) + drho;
    const T vx = jx / r, vy = jy / r;
    const T th = T(d.theta);
    const T hx[3] = {T(0.5) * (th + vx * vx - vx), T(1) - th - vx * vx, T(0.5) * (th + vx * vx + vx)};
    const T hy[3] = {T(0.5) * (th + vy * vy - vy), T(1) - th - vy * vy, T(0.5) * (th + vy * vy + vy)};
    const T gx[3] = {vx - T(0.5), T(-2) * vx, vx + T(0.5)};
    const T gy[3] = {vy - T(0.5), T(-2) * vy, vy + T(0.5)};
    T ax = T(0), ay = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int a = cx(i) + 1, b = cy(i) + 1;
      const T fb = fbar[local_index(i, q, y, d)];
      ax += fb * r * gx[a] * hy[b];
      ay += fb * r * hx[a] * gy[b];
    }
    sh[0][w][lane] = ax;
    sh[1][w][lane] = ay;
  }
  __syncthreads();
  if (tl.xt >= 0) {
    const int64_t n = int64_t(y) * d.nx + tl.xt;
    uxb[n] = sh[0][tl.jt][tl.lt];
    uyb[n] = sh[1][tl.jt][tl.lt];
  }
}

// --- step dispatch ---------------------------------------------------------------------------

template <class S, int MODEL, int NPT, bool WT>
hipError_t launch_step_w(const RunDesc& d, int phase, const void* src, void* dst, void* rec, hipStream_t st) {
  using T = typename StorageTraits<S>::T;
  const Geo g = make_geo(d, NPT);
  const Coef<T> k = make_coef<T>(d);
  const S* s = static_cast<const S*>(src);
  S* o = static_cast<S*>(dst);
  T* r = static_cast<T*>(rec);
  const dim3 grid = step_grid(g), block(kBlock);
  if (rec) {
    if (phase == PH_AB) hipLaunchKernelGGL((k_step<S, MODEL, PH_AB, true, NPT, WT>), grid, block, 0, st, s, o, g, k, r, d.rs_rec);
    else if (phase == PH_AA_EVEN) hipLaunchKernelGGL((k_step<S, MODEL, PH_AA_EVEN, true, NPT, WT>), grid, block, 0, st, s, o, g, k, r, d.rs_rec);
    else hipLaunchKernelGGL((k_step<S, MODEL, PH_AA_ODD, true, NPT, WT>), grid, block, 0, st, s, o, g, k, r, d.rs_rec);
  } else {
    if (phase == PH_AB) hipLaunchKernelGGL((k_step<S, MODEL, PH_AB, false, NPT, WT>), grid, block, 0, st, s, o, g, k, r, d.rs_rec);
    else if (phase == PH_AA_EVEN) hipLaunchKernelGGL((k_step<S, MODEL, PH_AA_EVEN, false, NPT, WT>), grid, block, 0, st, s, o, g, k, r, d.rs_rec);
    else hipLaunchKernelGGL((k_step<S, MODEL, PH_AA_ODD, false, NPT, WT>), grid, block, 0, st, s, o, g, k, r, d.rs_rec);
  }
  return hipGetLastError();
}

template <class S, int MODEL, int NPT>
hipError_t launch_step_n(const RunDesc& d, int phase, const void* src, void* dst, void* rec, hipStream_t st) {
  return d.wt_stores ? launch_step_w<S, MODEL, NPT, true>(d, phase, src, dst, rec, st)
                     : launch_step_w<S, MODEL, NPT, false>(d, phase, src, dst, rec, st);
}

// Nodes per thread of the step kernel. Two or four nodes per thread put more loads in flight
// before the first collision, which pays where the collision is long relative to the bytes
// moved (16-bit storage); the FP32 and FP64 paths are bandwidth-bound and run fastest with one.
// Measured on MI355X, 8192^2, complete model (GLUPS, 1/2/4 nodes per thread): FP16
// 148/160/167, BF16 149/168/168, FP32 90.6/82.6/81.0; LBGK FP16 176/178/168.
template <class S> struct NodesPerThread { static constexpr int oreg = 1, bgk = 1; };
template <> struct NodesPerThread<_Float16> { static constexpr int oreg = 4, bgk = 2; };
template <> struct NodesPerThread<bf16_t> { static constexpr int oreg = 2, bgk = 2; };

template <class S, int MODEL>
hipError_t launch_step_m(const RunDesc& d, int phase, const void* src, void* dst, void* rec, hipStream_t st) {
  constexpr int npt = MODEL == M_BGK ? NodesPerThread<S>::bgk : NodesPerThread<S>::oreg;
  // A wavefront's NPT groups must all lie inside the row or all past it.
  if constexpr (npt > 1) {
    if ((d.pitch / kLanes) % (npt * kBlock / kLanes) == 0)
      return launch_step_n<S, MODEL, npt>(d, phase, src, dst, rec, st);
  }
  return launch_step_n<S, MODEL, 1>(d, phase, src, dst, rec, st);
}

template <class S, int MODEL>
hipError_t launch_step_walls(const RunDesc& d, const void* src, void* dst, hipStream_t st) {
  using T = typename StorageTraits<S>::T;
  const Geo g = make_geo(d, 1);
  hipLaunchKernelGGL((k_step_walls<S, MODEL>), step_grid(g), dim3(kBlock), 0, st, static_cast<const S*>(src),
                     static_cast<S*>(dst), g, make_coef<T>(d));
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::step(const RunDesc& d, int phase, const void* src, void* dst, void* rec, hipStream_t st) {
  if (d.walls) {
    if (phase != PH_AB || rec) return hipErrorInvalidValue;
    switch (d.model) {
      case M_BGK: return launch_step_walls<S, M_BGK>(d, src, dst, st);
      case M_UC: return launch_step_walls<S, M_UC>(d, src, dst, st);
      case M_PARTIAL: return launch_step_walls<S, M_PARTIAL>(d, src, dst, st);
      default: return launch_step_walls<S, M_COMPLETE>(d, src, dst, st);
    }
  }
  switch (d.model) {
    case M_BGK: return launch_step_m<S, M_BGK>(d, phase, src, dst, rec, st);
    case M_UC: return launch_step_m<S, M_UC>(d, phase, src, dst, rec, st);
    case M_PARTIAL: return launch_step_m<S, M_PARTIAL>(d, phase, src, dst, rec, st);
    default: return launch_step_m<S, M_COMPLETE>(d, phase, src, dst, rec, st);
  }
}

template <class S, int MODEL>
hipError_t launch_step2_m(const RunDesc& d, const void* src, void* dst, void* rec1, void* rec2, hipStream_t st) {
  using T = typename StorageTraits<S>::T;
  const Geo g = make_geo(d, 1);
  const Coef<T> k = make_coef<T>(d);
  const dim3 grid(unsigned(g.S / kFuseGroups), unsigned(d.fuse_rb));
  const dim3 block((kFuseGroups + 2) * kLanes);
  const S* s = static_cast<const S*>(src);
  S* o = static_cast<S*>(dst);
  T* r1 = static_cast<T*>(rec1);
  T* r2 = static_cast<T*>(rec2);
  if (rec1 && rec2) {
    if (d.wt_stores) hipLaunchKernelGGL((k_step2<S, MODEL, true, true>), grid, block, 0, st, s, o, g, k, r1, r2, d.rs_rec);
    else hipLaunchKernelGGL((k_step2<S, MODEL, true, false>), grid, block, 0, st, s, o, g, k, r1, r2, d.rs_rec);
  } else {
    if (d.wt_stores) hipLaunchKernelGGL((k_step2<S, MODEL, false, true>), grid, block, 0, st, s, o, g, k, r1, r2, d.rs_rec);
    else hipLaunchKernelGGL((k_step2<S, MODEL, false, false>), grid, block, 0, st, s, o, g, k, r1, r2, d.rs_rec);
  }
  return hipGetLastError();
}

// Row blocks of the two-step kernel. A block of h rows computes h + 2 rows of step 1 and h
// of step 2, and a compute unit works through its share of the blocks in turn, so a launch
// takes about ceil(blocks / CUs) (2 h + 2) row-steps of one block, h the tallest block.
// The planner takes the row-block count of least such cost with blocks of kFuseMinRows to
// kFuseRows rows (ties: the taller blocks); for each count of blocks per compute unit only
// the largest row-block count that keeps it needs checking. On MI355X this ranking matched
// the measured throughput of every candidate tried on 512^2 to 4096^2 grids. In mode 0 a
// grid that cannot give three quarters of the compute units a block keeps single steps.
// The two-step adjoint kernel has the same block structure and uses the same plan.
// Least-cost row-block count for blocks of kFuseMinRows to max_rows rows (0: none).
inline long plan_rows(long ny, long cols, long cus, long max_rows) {
  const long nb_lo = (ny + max_rows - 1) / max_rows;
  const long nb_hi = std::min(std::max(nb_lo, ny / kFuseMinRows), 65535L);
  if (nb_lo > nb_hi) return 0;
  long best = 0, best_cost = 0;
  const long w0 = std::max(1L, (cols * nb_lo + cus - 1) / cus);
  for (long w = w0; w < w0 + 4096; ++w) {
    const long nb = std::min(nb_hi, std::max(nb_lo, w * cus / cols));
    const long rows = (ny + nb - 1) / nb;
    const long cost = (cols * nb + cus - 1) / cus * (2 * rows + 2);
    if (best == 0 || cost < best_cost) best = nb, best_cost = cost;
    if (nb == nb_hi) break;
  }
  return best;
}

// tall: also consider blocks of up to kFuseRowsTall rows, taken when the grid then gives every
// block a compute unit of its own (one round of blocks).
inline int plan_row_blocks(const RunDesc& d, int mode, bool tall) {
  if (d.nx % kLanes != 0 || (d.pitch / kLanes) % kFuseGroups != 0) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return 0;
  const long cols = d.pitch / kLanes / kFuseGroups;
  long best = plan_rows(d.ny, cols, cus, kFuseRows);
  if (tall) {
    const long t = plan_rows(d.ny, cols, cus, kFuseRowsTall);
    if (t > 0 && cols * t <= cus) best = t;
  }
  if (best == 0 || (mode == 0 && 4 * cols * best < 3L * cus)) return 0;
  return int(best);
}

template <class S>
int Engine<S>::fuse_row_blocks(const RunDesc& d, int mode) {
  return plan_row_blocks(d, mode, FuseTall<S>::value);
}

template <class S>
int Engine<S>::adjoint_row_blocks(const RunDesc& d, int mode) {
  return plan_row_blocks(d, mode, FuseTall<T>::value);
}

template <class S>
hipError_t Engine<S>::step2(const RunDesc& d, const void* src, void* dst, void* rec1, void* rec2, hipStream_t st) {
  if (d.fuse_rb < 1 || d.fuse_rb > d.ny) return hipErrorInvalidValue;
  switch (d.model) {
    case M_BGK: return launch_step2_m<S, M_BGK>(d, src, dst, rec1, rec2, st);
    case M_UC: return launch_step2_m<S, M_UC>(d, src, dst, rec1, rec2, st);
    case M_PARTIAL: return launch_step2_m<S, M_PARTIAL>(d, src, dst, rec1, rec2, st);
    default: return launch_step2_m<S, M_COMPLETE>(d, src, dst, rec1, rec2, st);
  }
}

template <class S>
hipError_t Engine<S>::init(const RunDesc& d, LayoutSel L, void* buf, const double* rho, const double* ux,
                           const double* uy, hipStream_t st) {
  hipLaunchKernelGGL(k_init<S>, tile_grid(d), dim3(kBlock), 0, st, static_cast<S*>(buf), d, L, rho, ux, uy);
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::get(const RunDesc& d, LayoutSel L, const void* buf, bool out_f64, void* out, hipStream_t st) {
  if (out_f64)
    hipLaunchKernelGGL((k_get<S, double>), tile_grid(d), dim3(kBlock), 0, st, static_cast<const S*>(buf), d, L,
                       static_cast<double*>(out));
  else
    hipLaunchKernelGGL((k_get<S, float>), tile_grid(d), dim3(kBlock), 0, st, static_cast<const S*>(buf), d, L,
                       static_cast<float*>(out));
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::set(const RunDesc& d, LayoutSel L, void* buf, const double* in, hipStream_t st) {
  hipLaunchKernelGGL(k_set<S>, tile_grid(d), dim3(kBlock), 0, st, static_cast<S*>(buf), d, L, in);
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::moments(const RunDesc& d, LayoutSel L, const void* buf, bool out_f64, void* rho, void* ux,
                              void* uy, hipStream_t st) {
  if (out_f64)
    hipLaunchKernelGGL((k_moments<S, double>), tile_grid(d), dim3(kBlock), 0, st, static_cast<const S*>(buf), d,
                       L, static_cast<double*>(rho), static_cast<double*>(ux), static_cast<double*>(uy));
  else
    hipLaunchKernelGGL((k_moments<S, float>), tile_grid(d), dim3(kBlock), 0, st, static_cast<const S*>(buf), d,
                       L, static_cast<float*>(rho), static_cast<float*>(ux), static_cast<float*>(uy));
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::invariants(const RunDesc& d, LayoutSel L, const void* buf, double* partial, double* result,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partial<S>, dim3(kReduceBlocks), dim3(kBlock), 0, st, static_cast<const S*>(buf), d, L,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final<S>, dim3(1), dim3(kBlock), 0, st, partial, kReduceBlocks,
                     d.rho0 * double(d.nx) * double(d.ny), result);
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::seed(const RunDesc& d, LayoutSel L, const void* buf, const T* rhob, const T* uxb, const T* uyb,
                           T* fbar, hipStream_t st) {
  hipLaunchKernelGGL((k_seed<S, T>), tile_grid(d), dim3(kBlock), 0, st, static_cast<const S*>(buf), d, L, rhob, uxb,
                     uyb, fbar);
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::fbar_import(const RunDesc& d, const T* dense, T* fbar, hipStream_t st) {
  hipLaunchKernelGGL(k_fbar_import<T>, dim3(node_blocks(d)), dim3(kBlock), 0, st, d, dense, fbar);
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::fbar_export(const RunDesc& d, const T* fbar, T* dense, hipStream_t st) {
  hipLaunchKernelGGL(k_fbar_export<T>, dim3(node_blocks(d)), dim3(kBlock), 0, st, d, fbar, dense);
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::adjoint_step2(const RunDesc& d, const T* fbar_next, T* fbar, const T* rec_hi, const T* rec_lo,
                                    hipStream_t st) {
  if (d.adj_rb < 1 || d.adj_rb > d.ny) return hipErrorInvalidValue;
  const Geo g = make_geo(d, 1);
  const Coef<T> k = make_coef<T>(d);
  const dim3 grid(unsigned(g.S / kFuseGroups), unsigned(d.adj_rb)), block((kFuseGroups + 2) * kLanes);
  switch (d.model) {
    case M_BGK: hipLaunchKernelGGL((k_adjoint_step2<T, M_BGK>), grid, block, 0, st, fbar_next, fbar, g, k, rec_hi, rec_lo, d.rs_rec); break;
    case M_UC: hipLaunchKernelGGL((k_adjoint_step2<T, M_UC>), grid, block, 0, st, fbar_next, fbar, g, k, rec_hi, rec_lo, d.rs_rec); break;
    case M_PARTIAL: hipLaunchKernelGGL((k_adjoint_step2<T, M_PARTIAL>), grid, block, 0, st, fbar_next, fbar, g, k, rec_hi, rec_lo, d.rs_rec); break;
    default: hipLaunchKernelGGL((k_adjoint_step2<T, M_COMPLETE>), grid, block, 0, st, fbar_next, fbar, g, k, rec_hi, rec_lo, d.rs_rec); break;
  }
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::adjoint_step(const RunDesc& d, const T* fbar_next, T* fbar, const T* rec, hipStream_t st) {
  const Geo g = make_geo(d, 1);
  const Coef<T> k = make_coef<T>(d);
  const dim3 grid = step_grid(g), block(kBlock);
  switch (d.model) {
    case M_BGK: hipLaunchKernelGGL((k_adjoint_step<T, M_BGK>), grid, block, 0, st, fbar_next, fbar, g, k, rec, d.rs_rec); break;
    case M_UC: hipLaunchKernelGGL((k_adjoint_step<T, M_UC>), grid, block, 0, st, fbar_next, fbar, g, k, rec, d.rs_rec); break;
    case M_PARTIAL: hipLaunchKernelGGL((k_adjoint_step<T, M_PARTIAL>), grid, block, 0, st, fbar_next, fbar, g, k, rec, d.rs_rec); break;
    default: hipLaunchKernelGGL((k_adjoint_step<T, M_COMPLETE>), grid, block, 0, st, fbar_next, fbar, g, k, rec, d.rs_rec); break;
  }
  return hipGetLastError();
}

template <class S>
hipError_t Engine<S>::ic_adjoint(const RunDesc& d, LayoutSel L, const void* buf0, const T* fbar, T* uxb, T* uyb,
                                 hipStream_t st) {
  hipLaunchKernelGGL((k_ic_adjoint<S, T>), tile_grid(d), dim3(kBlock), 0, st, static_cast<const S*>(buf0), d, L, fbar,
                     uxb, uyb);
  return hipGetLastError();
}

}  // namespace lbm
