// Fused stream + collide kernel of the D2Q9 OReg-GEq step over a structure-of-arrays
// population layout, and the adjoint step kernel. Instantiated per storage type in
// step_<type>.hip.
//
// Data layout (HBM): nine planes of shifted populations g_i, plane i at byte offset
// i * plane * sizeof(S), each plane ny rows of `pitch` elements (pitch = nx rounded up to 8,
// so every row starts 16-byte aligned). One thread updates VEC consecutive nodes of one
// row (VEC * sizeof(S) = 16 bytes: one aligned vector load per population), 256 threads
// per block, blocks remapped so that consecutive tiles land on the same XCD.
//
// Streaming patterns. The state at time n satisfies f_i^n(x) = buf[s(i)][x - d c_i]:
//   A-B:       d = 1, s(i) = i (the buffer holds post-collision values at their origin;
//              the step pulls from x - c_i and writes in place in the other buffer).
//   AA, even:  d = 0, s(i) = i; the step reads locally and writes f*_i to slot opp(i).
//   AA, odd:   d = 1, s(i) = opp(i); the step pulls and pushes f*_i to x + c_i, slot i.
// Each AA step reads and writes exactly the same set of locations per node, so one buffer
// suffices and threads never race.
#pragma once

#include <type_traits>

#include "lbm_device.h"

namespace lbm {

constexpr int kBlock = 256;

struct Geo {
  int nx, ny, pitch;
  int64_t plane;   // elements between population planes
  int ngx;         // thread groups per row = ceil(nx / VEC)
  int ngroups;     // ngx * ny
  int nblocks;     // ceil(ngroups / kBlock)
  int nb8;         // ceil(nblocks / 8): blocks per XCD
};

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <class S, int VEC>
struct alignas(sizeof(S) * VEC) Pack {
  S v[VEC];
};

__device__ __forceinline__ int wrapx(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// Load the values a row holds at x0 + k + DX, k = 0..VEC-1 (periodic in x).
// Full groups use one aligned vector load plus, for DX = +-1, one element of the
// neighbouring group; the ragged tail of a row falls back to element loads.
template <class S, int VEC, int DX, class T>
__device__ __forceinline__ void load_row(const S* row, int x0, int nx, bool full, T out[VEC]) {
  using Tr = StorageTraits<S>;
  if (full) {
    Pack<S, VEC> a;
    if constexpr (DX == 0 || VEC > 1) a = *reinterpret_cast<const Pack<S, VEC>*>(row + x0);
    if constexpr (DX == 0) {
#pragma unroll
      for (int k = 0; k < VEC; ++k) out[k] = Tr::load(a.v[k]);
    } else if constexpr (DX < 0) {
#pragma unroll
      for (int k = 1; k < VEC; ++k) out[k] = Tr::load(a.v[k - 1]);
      out[0] = Tr::load(row[x0 == 0 ? nx - 1 : x0 - 1]);
    } else {
#pragma unroll
      for (int k = 0; k + 1 < VEC; ++k) out[k] = Tr::load(a.v[k + 1]);
      out[VEC - 1] = Tr::load(row[x0 + VEC == nx ? 0 : x0 + VEC]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      const int x = min(x0 + k, nx - 1);
      out[k] = Tr::load(row[wrapx(x + DX, nx)]);
    }
  }
}

// Store val[k] to x0 + k + DX (periodic in x), k = 0..VEC-1, nodes x0 + k < nx only.
template <class S, int VEC, int DX, class T>
__device__ __forceinline__ void store_row(S* row, int x0, int nx, bool full, const T val[VEC]) {
  using Tr = StorageTraits<S>;
  if constexpr (DX == 0) {
    if (full) {
      Pack<S, VEC> p;
#pragma unroll
      for (int k = 0; k < VEC; ++k) p.v[k] = Tr::store(val[k]);
      *reinterpret_cast<Pack<S, VEC>*>(row + x0) = p;
    } else {
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        if (x0 + k < nx) row[x0 + k] = Tr::store(val[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k)
      if (full || x0 + k < nx) row[wrapx(x0 + k + DX, nx)] = Tr::store(val[k]);
  }
}

// Thread -> (row, first node) with the XCD-aware block remap. Returns false for idle threads.
__device__ __forceinline__ bool map_thread(const Geo& geo, int vec, int& y, int& x0) {
  const int b = blockIdx.x;
  const int L = (b & 7) * geo.nb8 + (b >> 3);
  if (L >= geo.nblocks) return false;
  const int gid = L * kBlock + int(threadIdx.x);
  if (gid >= geo.ngroups) return false;
  y = gid / geo.ngx;
  x0 = (gid - y * geo.ngx) * vec;
  return true;
}

// One time step for VEC nodes per thread. src and dst alias in the AA phases.
template <class S, int VEC, int MODEL, int PH, bool REC>
__global__ void __launch_bounds__(kBlock)
k_step(const S* src, S* dst, Geo geo, Coef<typename StorageTraits<S>::T> k,
       typename StorageTraits<S>::T* rec, int64_t rec_plane) {
  using T = typename StorageTraits<S>::T;
  int y, x0;
  if (!map_thread(geo, VEC, y, x0)) return;
  const bool full = x0 + VEC <= geo.nx;
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;

  T g[Q][VEC];
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr bool shift = (PH != PH_AA_EVEN);
    constexpr int slot = (PH == PH_AA_ODD) ? opp(i) : i;
    constexpr int dx = shift ? -cx(i) : 0;
    constexpr int dy = shift ? -cy(i) : 0;
    const int yy = dy < 0 ? ym : (dy > 0 ? yp : y);
    load_row<S, VEC, dx>(src + slot * geo.plane + int64_t(yy) * geo.pitch, x0, geo.nx, full, g[i]);
  });

  T out[Q][VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    T gv[Q], ov[Q], rv[NREC];
#pragma unroll
    for (int i = 0; i < Q; ++i) gv[i] = g[i][v];
    collide<T, MODEL>(gv, ov, k, REC ? rv : nullptr);
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i][v] = ov[i];
    if constexpr (REC) {
#pragma unroll
      for (int r = 0; r < NREC; ++r) g[r][v] = rv[r];  // reuse registers for the record
    }
  }
  if constexpr (REC) {
#pragma unroll
    for (int r = 0; r < NREC; ++r)
      store_row<T, VEC, 0>(rec + r * rec_plane + int64_t(y) * geo.pitch, x0, geo.nx, full, g[r]);
  }

  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr bool shift = (PH == PH_AA_ODD);
    constexpr int slot = (PH == PH_AA_EVEN) ? opp(i) : i;
    constexpr int dx = shift ? cx(i) : 0;
    constexpr int dy = shift ? cy(i) : 0;
    const int yy = dy < 0 ? ym : (dy > 0 ? yp : y);
    store_row<S, VEC, dx>(dst + slot * geo.plane + int64_t(yy) * geo.pitch, x0, geo.nx, full, out[i]);
  });
}

// One reverse step of the discrete adjoint: fbar^n(x) = J(m^n(x))^T fbar*(x) with the
// reverse-streamed fbar*_i(x) = fbar^{n+1}_i(x + c_i). fbar planes are natural-layout
// compute-type planes with the same pitch; rec holds the step's recorded moments.
template <class T, int VEC, int MODEL>
__global__ void __launch_bounds__(kBlock)
k_adjoint_step(const T* __restrict__ fbar_next, T* __restrict__ fbar, Geo geo, Coef<T> k,
               const T* __restrict__ rec, int64_t rec_plane) {
  int y, x0;
  if (!map_thread(geo, VEC, y, x0)) return;
  const bool full = x0 + VEC <= geo.nx;
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;
  T a[Q][VEC];
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int dx = cx(i), dy = cy(i);
    const int yy = dy < 0 ? ym : (dy > 0 ? yp : y);
    load_row<T, VEC, dx>(fbar_next + i * geo.plane + int64_t(yy) * geo.pitch, x0, geo.nx, full, a[i]);
  });
  T m[NREC][VEC];
#pragma unroll
  for (int r = 0; r < NREC; ++r) load_row<T, VEC, 0>(rec + r * rec_plane + int64_t(y) * geo.pitch, x0, geo.nx, full, m[r]);
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    T fs[Q], rv[NREC], fb[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) fs[i] = a[i][v];
#pragma unroll
    for (int r = 0; r < NREC; ++r) rv[r] = m[r][v];
    collide_vjp<T, MODEL>(fs, rv, k, fb);
#pragma unroll
    for (int i = 0; i < Q; ++i) a[i][v] = fb[i];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) store_row<T, VEC, 0>(fbar + i * geo.plane + int64_t(y) * geo.pitch, x0, geo.nx, full, a[i]);
}

}  // namespace lbm
