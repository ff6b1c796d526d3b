// Fused stream + collide kernel of the D2Q9 OReg-GEq step and the adjoint step kernel.
// Instantiated per storage type in step_<type>.hip.
//
// Data layout (HBM): shifted populations g_i, row-interleaved structure of arrays: element
// (i, x, y) sits at y * rs + i * ps + x with ps = pitch (nx rounded up to 8, so every
// population row starts 16-byte aligned) and rs = 9 * pitch. The nine population rows of a
// lattice row are contiguous, which keeps the 18 concurrent read/write streams of a step
// within a compact address window (measured on MI355X: 6.4 TB/s for the 9-in/9-out
// skeleton, against 5.6 TB/s with nine separate planes). Loads and stores are
// nontemporal: every population is read once and written once per step.
//
// One thread updates VEC consecutive nodes of one row (one aligned vector load per
// population); a block of 256 threads covers one segment of one row, so the row, its two
// periodic neighbours and every row/population base address are uniform (scalar
// registers) and each lane only adds its 32-bit in-row offset.
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

constexpr int kRowsY = 32768;  // rows per grid y-dimension slice

struct Geo {
  int nx, ny;
  int ps;          // elements between the rows of two populations of one lattice row
  int64_t rs;      // elements between two lattice rows
  int nseg;        // blocks per lattice row = ceil(ceil(nx / VEC) / kBlock)
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

// Element type the nontemporal builtins accept, and its native vector of VEC lanes.
template <class S> struct Bits { using type = S; };
template <> struct Bits<bf16_t> { using type = uint16_t; };
template <class E, int N> struct NVec { typedef E type __attribute__((ext_vector_type(N))); };
template <class E> struct NVec<E, 1> { using type = E; };

template <class S, int VEC>
__device__ __forceinline__ Pack<S, VEC> ld_nt(const S* p) {
  using V = typename NVec<typename Bits<S>::type, VEC>::type;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  Pack<S, VEC> r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

template <class S, int VEC>
__device__ __forceinline__ void st_nt(S* p, const Pack<S, VEC>& r) {
  using V = typename NVec<typename Bits<S>::type, VEC>::type;
  V v;
  __builtin_memcpy(&v, &r, sizeof(r));
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}

template <class S>
__device__ __forceinline__ S ld1(const S* p) { return ld_nt<S, 1>(p).v[0]; }

template <class S>
__device__ __forceinline__ void st1(S* p, S v) {
  Pack<S, 1> r;
  r.v[0] = v;
  st_nt<S, 1>(p, r);
}

__device__ __forceinline__ int wrapx(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// Element x of a population row: base (uniform: buffer + row + population) plus the
// lane's 32-bit byte offset.
template <class S>
__device__ __forceinline__ const S* at(const char* base, int x) {
  return reinterpret_cast<const S*>(base + uint32_t(x) * uint32_t(sizeof(S)));
}
template <class S>
__device__ __forceinline__ S* at(char* base, int x) {
  return reinterpret_cast<S*>(base + uint32_t(x) * uint32_t(sizeof(S)));
}

// Load the values a population row holds at x0 + k + DX, k = 0..VEC-1 (periodic in x).
// Full groups use one aligned vector load plus, for DX = +-1, one element of the
// neighbouring group; the ragged tail of a row uses element loads.
template <class S, int VEC, int DX, class T>
__device__ __forceinline__ void load_row(const char* base, int x0, int nx, bool full, T out[VEC]) {
  using Tr = StorageTraits<S>;
  if (full) {
    Pack<S, VEC> a;
    if constexpr (DX == 0 || VEC > 1) a = ld_nt<S, VEC>(at<S>(base, x0));
    if constexpr (DX == 0) {
#pragma unroll
      for (int k = 0; k < VEC; ++k) out[k] = Tr::load(a.v[k]);
    } else if constexpr (DX < 0) {
#pragma unroll
      for (int k = 1; k < VEC; ++k) out[k] = Tr::load(a.v[k - 1]);
      out[0] = Tr::load(ld1(at<S>(base, x0 == 0 ? nx - 1 : x0 - 1)));
    } else {
#pragma unroll
      for (int k = 0; k + 1 < VEC; ++k) out[k] = Tr::load(a.v[k + 1]);
      out[VEC - 1] = Tr::load(ld1(at<S>(base, x0 + VEC == nx ? 0 : x0 + VEC)));
    }
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k) out[k] = Tr::load(ld1(at<S>(base, wrapx(min(x0 + k, nx - 1) + DX, nx))));
  }
}

// Store val[k] to x0 + k + DX (periodic in x), k = 0..VEC-1, nodes x0 + k < nx only.
template <class S, int VEC, int DX, class T>
__device__ __forceinline__ void store_row(char* base, int x0, int nx, bool full, const T val[VEC]) {
  using Tr = StorageTraits<S>;
  if constexpr (DX == 0) {
    if (full) {
      Pack<S, VEC> p;
#pragma unroll
      for (int k = 0; k < VEC; ++k) p.v[k] = Tr::store(val[k]);
      st_nt<S, VEC>(at<S>(base, x0), p);
    } else {
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        if (x0 + k < nx) st1(at<S>(base, x0 + k), Tr::store(val[k]));
    }
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k)
      if (full || x0 + k < nx) st1(at<S>(base, wrapx(x0 + k + DX, nx)), Tr::store(val[k]));
  }
}

// Block -> lattice row (uniform), thread -> first node of its group. Grid:
// (nseg, min(ny, kRowsY), ceil(ny / kRowsY)).
__device__ __forceinline__ bool map_thread(const Geo& geo, int vec, int& y, int& x0) {
  y = int(blockIdx.z) * kRowsY + int(blockIdx.y);
  x0 = (int(blockIdx.x) * kBlock + int(threadIdx.x)) * vec;
  return y < geo.ny && x0 < geo.nx;
}

// One time step for VEC nodes per thread. src and dst alias in the AA phases. With REC the
// moments (rho, u_x, u_y, N_xx, N_xy) of every node are written to rec, laid out like the
// populations with five entries per lattice row (row stride rec_rs).
template <class S, int VEC, int MODEL, int PH, bool REC>
__global__ void __launch_bounds__(kBlock)
k_step(const S* src, S* dst, Geo geo, Coef<typename StorageTraits<S>::T> k,
       typename StorageTraits<S>::T* rec, int64_t rec_rs) {
  using T = typename StorageTraits<S>::T;
  int y, x0;
  if (!map_thread(geo, VEC, y, x0)) return;
  const bool full = x0 + VEC <= geo.nx;
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;
  const size_t rsb = size_t(geo.rs) * sizeof(S), psb = size_t(geo.ps) * sizeof(S);
  const char* sr[3] = {reinterpret_cast<const char*>(src) + ym * rsb, reinterpret_cast<const char*>(src) + y * rsb,
                       reinterpret_cast<const char*>(src) + yp * rsb};
  char* dr[3] = {reinterpret_cast<char*>(dst) + ym * rsb, reinterpret_cast<char*>(dst) + y * rsb,
                 reinterpret_cast<char*>(dst) + yp * rsb};

  T g[Q][VEC];
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr bool shift = (PH != PH_AA_EVEN);
    constexpr int slot = (PH == PH_AA_ODD) ? opp(i) : i;
    constexpr int dx = shift ? -cx(i) : 0;
    constexpr int dy = shift ? -cy(i) : 0;
    load_row<S, VEC, dx>(sr[dy + 1] + slot * psb, x0, geo.nx, full, g[i]);
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
    char* rrow = reinterpret_cast<char*>(rec) + y * (size_t(rec_rs) * sizeof(T));
#pragma unroll
    for (int r = 0; r < NREC; ++r) store_row<T, VEC, 0>(rrow + r * size_t(geo.ps) * sizeof(T), x0, geo.nx, full, g[r]);
  }

  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr bool shift = (PH == PH_AA_ODD);
    constexpr int slot = (PH == PH_AA_EVEN) ? opp(i) : i;
    constexpr int dx = shift ? cx(i) : 0;
    constexpr int dy = shift ? cy(i) : 0;
    store_row<S, VEC, dx>(dr[dy + 1] + slot * psb, x0, geo.nx, full, out[i]);
  });
}

// One reverse step of the discrete adjoint: fbar^n(x) = J(m^n(x))^T fbar*(x) with the
// reverse-streamed fbar*_i(x) = fbar^{n+1}_i(x + c_i). fbar uses the population layout in
// the compute type (geo describes it); rec holds the step's recorded moments.
template <class T, int VEC, int MODEL>
__global__ void __launch_bounds__(kBlock)
k_adjoint_step(const T* __restrict__ fbar_next, T* __restrict__ fbar, Geo geo, Coef<T> k,
               const T* __restrict__ rec, int64_t rec_rs) {
  int y, x0;
  if (!map_thread(geo, VEC, y, x0)) return;
  const bool full = x0 + VEC <= geo.nx;
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;
  const size_t rsb = size_t(geo.rs) * sizeof(T), psb = size_t(geo.ps) * sizeof(T);
  const char* nr[3] = {reinterpret_cast<const char*>(fbar_next) + ym * rsb,
                       reinterpret_cast<const char*>(fbar_next) + y * rsb,
                       reinterpret_cast<const char*>(fbar_next) + yp * rsb};
  T a[Q][VEC];
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    load_row<T, VEC, cx(i)>(nr[cy(i) + 1] + i * psb, x0, geo.nx, full, a[i]);
  });
  T m[NREC][VEC];
  const char* rrow = reinterpret_cast<const char*>(rec) + y * (size_t(rec_rs) * sizeof(T));
#pragma unroll
  for (int r = 0; r < NREC; ++r) load_row<T, VEC, 0>(rrow + r * psb, x0, geo.nx, full, m[r]);
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
  char* orow = reinterpret_cast<char*>(fbar) + y * rsb;
#pragma unroll
  for (int i = 0; i < Q; ++i) store_row<T, VEC, 0>(orow + i * psb, x0, geo.nx, full, a[i]);
}

}  // namespace lbm
