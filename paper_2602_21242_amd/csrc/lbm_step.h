// Fused stream + collide kernel of the D2Q9 OReg-GEq step and the adjoint step kernel.
// Instantiated per storage type in step_<type>.hip.
//
// Data layout (HBM): shifted populations g_i, row-interleaved structure of arrays: element
// (i, x, y) sits at y * rs + i * ps + pos(x) with ps = pitch = 64 S, S = ceil(nx / 64),
// rs = 9 * pitch. Within a row the nodes are lane-strided: node x = lane * S + s is stored at
// pos(x) = 64 s + lane, so the 64 lanes of a wave hold the nodes s, s + S, ..., s + 63 S.
// The x-neighbours of those nodes (s - 1 and s + 1 of the same lanes) are again one whole,
// aligned 64-element group, so the streaming step's x-shifts cost no extra cache lines; only
// the groups s = 0 and s = S - 1 read a group rotated by one lane. (With contiguous rows
// every x-shifted wave load straddles one more cache line, which measured 5-7 % slower on
// MI355X for the 9-in/9-out pull.) The nine population rows of a lattice row are contiguous,
// which keeps the 18 concurrent read/write streams of a step within a compact address
// window. Loads and stores are nontemporal: every population is read once and written once
// per step. Rows are padded to whole groups; padding positions (x >= nx, last lanes only)
// are never read by a real node. The step kernel lets a padding lane read and write its own
// padding slot (no per-lane guards), the other kernels skip padding.
//
// One thread updates NPT nodes (one lane of NPT consecutive groups); a block of 256 threads
// covers 4 NPT groups of one row, so the row, its two periodic neighbours and every
// row/population base address are uniform (scalar registers) and each lane only adds its
// 32-bit in-row offset.
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
constexpr int kLanes = 64;     // nodes per group of the lane-strided row layout (wavefront)
constexpr int kRowsY = 32768;  // rows per grid y-dimension slice

struct Geo {
  int nx, ny;
  int S;           // groups per row (pitch / 64)
  int ps;          // elements between the rows of two populations of one lattice row
  int64_t rs;      // elements between two lattice rows
  int nseg;        // blocks per lattice row = ceil(S / (4 NPT))
  int plast;       // pos(nx - 1)
};

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Element type the nontemporal builtins accept.
template <class S> struct Bits { using type = S; };
template <> struct Bits<bf16_t> { using type = uint16_t; };

template <class S>
__device__ __forceinline__ S ld1(const S* p) {
  using B = typename Bits<S>::type;
  const B b = __builtin_nontemporal_load(reinterpret_cast<const B*>(p));
  S r;
  __builtin_memcpy(&r, &b, sizeof(r));
  return r;
}

template <class S>
__device__ __forceinline__ void st1(S* p, S v) {
  using B = typename Bits<S>::type;
  B b;
  __builtin_memcpy(&b, &v, sizeof(b));
  __builtin_nontemporal_store(b, reinterpret_cast<B*>(p));
}

// A population load into the register form StorageTraits<S>::Raw (the storage type itself,
// or for FP16 its 16 bits zero-extended to 32).
// NT selects the nontemporal hint (the default) or a plain load.
template <class S, bool NT = true>
__device__ __forceinline__ typename StorageTraits<S>::Raw ld_raw(const S* p) {
  using R = typename StorageTraits<S>::Raw;
  using B = typename Bits<S>::type;
  if constexpr (std::is_same_v<R, S>) {
    if constexpr (NT) {
      return ld1(p);
    } else {
      const B b = *reinterpret_cast<const B*>(p);
      S r;
      __builtin_memcpy(&r, &b, sizeof(r));
      return r;
    }
  } else {
    static_assert(sizeof(S) == 2 && std::is_same_v<R, uint32_t>, "raw registers: 16-bit storage only");
    if constexpr (NT) return R(__builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p)));
    else return R(*reinterpret_cast<const uint16_t*>(p));
  }
}

// Element at in-row position p of a population row: base (uniform: buffer + row +
// population) plus the lane's 32-bit byte offset.
template <class S>
__device__ __forceinline__ const S* at(const char* base, int p) {
  return reinterpret_cast<const S*>(base + uint32_t(p) * uint32_t(sizeof(S)));
}
template <class S>
__device__ __forceinline__ S* at(char* base, int p) {
  return reinterpret_cast<S*>(base + uint32_t(p) * uint32_t(sizeof(S)));
}

// Buffer-resource accesses of the two-step forward kernel. One lattice row of a
// buffer (its nine population rows, or the five rows of a moment record) is described by a
// buffer resource in scalar registers, rebased to that row; an access adds the scalar offset
// of the population (or record entry) within the lattice row and the lane's 32-bit in-row
// byte offset, which stays in one vector register for the whole loop. (With plain pointers
// the compiler folded the loop-invariant lane offsets into nine 64-bit per-population
// addresses and added each row's offset to them in 64-bit vector arithmetic: 39 of the 333
// vector instructions of the FP32 two-step kernel's row loop; with buffer accesses and the
// scheduling fence of pair_sync the FP32 pair went from 142.6 to 150.1 GLUPS at 4096^2, FP16
// and BF16 from 183 to 189-190 at 8192^2.) The adjoint kernels keep plain pointers: the
// two-step adjoint ran 5 % slower with buffer accesses (433 against 414 us per launch at
// 4096^2), whatever its occupancy. Offsets within a lattice row stay below 2^31 bytes:
// lbm_init rejects wider rows.
constexpr int kRsrcWord3 = 0x00020000;  // resource word 3 of a raw buffer on the gfx9 family
constexpr int kAuxNT = 2;                // cache-policy operand of a nontemporal access (gfx950)
// Stores of the step kernels on grids whose population buffers exceed the last-level cache
// (WT, chosen by the host): nontemporal with the SC1 scope bit (device scope, written through
// rather than held in the XCD's L2). Measured on the FP32 two-step kernel, interleaved on one
// machine, us per launch: 210.5 -> 206.2 (4096^2), 832.0 -> 826.5 (8192^2); on another
// 212.3 -> 210.4 and 851.3 -> 841.8; the single-step kernel 186.8 -> 183.5 (4096^2). SC1
// without the nontemporal bit measured 3.5 % slower than plain nontemporal stores, stores
// without either hint 10 % slower, SC0 added to either no different; loads with SC1 no faster.
// On cache-resident grids SC1 costs instead: 1024^2 (38 MB per buffer) pair 18.1 -> 18.7 us,
// single step 14.2 -> 14.7, AA 13.4 -> 13.8, so there the stores stay plain nontemporal.
constexpr int kAuxStoreWT = kAuxNT | 16;
template <bool WT> constexpr int kAuxStore = WT ? kAuxStoreWT : kAuxNT;

struct RowRes {
  __amdgpu_buffer_rsrc_t r;
};

// Lattice row y of a buffer whose lattice rows are row_bytes apart.
__device__ __forceinline__ RowRes row_res(const void* buf, size_t row_bytes, int y) {
  char* base = const_cast<char*>(static_cast<const char*>(buf)) + size_t(y) * row_bytes;
  return RowRes{__builtin_amdgcn_make_buffer_rsrc(base, 0, int(uint32_t(row_bytes)), kRsrcWord3)};
}

// Element (soff + voff bytes into the lattice row) in the register form
// StorageTraits<E>::Raw for storage types, or as E itself for the compute types.
template <class E, bool NT>
__device__ __forceinline__ auto ldb(const RowRes& rr, int soff, uint32_t voff) {
  constexpr int aux = NT ? kAuxNT : 0;
  if constexpr (sizeof(E) == 8) {
    return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b64(rr.r, int(voff), soff, aux));
  } else if constexpr (sizeof(E) == 4) {
    return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b32(rr.r, int(voff), soff, aux));
  } else {
    const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(rr.r, int(voff), soff, aux);
    using R = typename StorageTraits<E>::Raw;
    if constexpr (std::is_same_v<R, uint32_t>) return uint32_t(h);
    else return __builtin_bit_cast(E, h);
  }
}

// Store of one element, nontemporal (every kernel writes each location once per launch), with
// the cache policy AUX.
template <class E, int AUX>
__device__ __forceinline__ void stb(const RowRes& rr, int soff, uint32_t voff, E v) {
  if constexpr (sizeof(E) == 8) {
    using V2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), rr.r, int(voff), soff, AUX);
  } else if constexpr (sizeof(E) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rr.r, int(voff), soff, AUX);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), rr.r, int(voff), soff, AUX);
  }
}

// In-row positions of a node and of its periodic x-neighbours.
struct RowPos {
  int p0, pm, pp;  // pos(x), pos(x - 1), pos(x + 1)
  template <int DX>
  __device__ __forceinline__ int of() const { return DX == 0 ? p0 : (DX < 0 ? pm : pp); }
};

// In-row positions of the node in group s at lane `lane` and of its periodic x-neighbours;
// false past the row (s >= S) and for padding.
__device__ __forceinline__ bool node_pos(const Geo& geo, int s, int lane, RowPos& r) {
  const int q = s * kLanes + lane;
  const int x = lane * geo.S + s;
  if (s >= geo.S || x >= geo.nx) return false;
  r.p0 = q;
  r.pm = s > 0 ? q - kLanes : (lane > 0 ? (geo.S - 1) * kLanes + lane - 1 : geo.plast);
  r.pp = x + 1 == geo.nx ? 0 : (s + 1 < geo.S ? q + kLanes : lane + 1);
  return true;
}

// Block -> lattice row (uniform); the block's wavefronts take NPT consecutive groups each,
// starting at the returned group s0. Grid: (nseg, min(ny, kRowsY), ceil(ny / kRowsY)) with
// nseg = ceil(S / (4 NPT)). A block is four 64-lane wavefronts, so s0 is uniform across a
// wavefront and is kept in a scalar register.
static_assert(kBlock % kLanes == 0, "a block must consist of whole 64-node groups");
template <int NPT>
__device__ __forceinline__ int first_group(int& y, int& lane) {
  y = int(blockIdx.z) * kRowsY + int(blockIdx.y);
  lane = int(threadIdx.x % kLanes);
  return (int(blockIdx.x) * (kBlock / kLanes) + __builtin_amdgcn_readfirstlane(int(threadIdx.x / kLanes))) * NPT;
}

// One time step; each thread updates NPT nodes (same lane, consecutive groups), issuing the
// loads of all of them before the first collision so that more memory traffic is in flight
// per wavefront. src and dst alias in the AA phases. With REC the moments (rho, u_x, u_y,
// N_xx, N_xy) of every node are written to rec, laid out like the populations with five
// entries per lattice row (row stride rec_rs).
template <class S, int MODEL, int PH, bool REC, int NPT, bool WT>
__global__ void __launch_bounds__(kBlock)
k_step(const S* src, S* dst, Geo geo, Coef<typename StorageTraits<S>::T> k,
       typename StorageTraits<S>::T* rec, int64_t rec_rs) {
  using T = typename StorageTraits<S>::T;
  using Tr = StorageTraits<S>;
  int y, lane;
  const int s0 = first_group<NPT>(y, lane);
  // Uniform exits only: the host launches NPT > 1 only when S is a multiple of 4 NPT, so a
  // wavefront's groups are either all inside the row or all past it. Padding lanes
  // (x >= nx) run on their own padding slot for every access (no real node reads those
  // slots and each still has one reader and one writer), so that all loads of the thread
  // stay in one basic block and are issued back to back.
  if (y >= geo.ny || s0 >= geo.S) return;
  RowPos rp[NPT];
#pragma unroll
  for (int n = 0; n < NPT; ++n)
    if (!node_pos(geo, s0 + n, lane, rp[n])) rp[n].p0 = rp[n].pm = rp[n].pp = (s0 + n) * kLanes + lane;
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;
  const size_t rsb = size_t(geo.rs) * sizeof(S), psb = size_t(geo.ps) * sizeof(S);
  const char* sr[3] = {reinterpret_cast<const char*>(src) + ym * rsb, reinterpret_cast<const char*>(src) + y * rsb,
                       reinterpret_cast<const char*>(src) + yp * rsb};
  // Stores through buffer descriptors of the three rows (cache policy kAuxStore<WT>).
  const RowRes dr[3] = {row_res(dst, rsb, ym), row_res(dst, rsb, y), row_res(dst, rsb, yp)};

  typename Tr::Raw gs[NPT][Q];
#pragma unroll
  for (int n = 0; n < NPT; ++n) {
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr bool shift = (PH != PH_AA_EVEN);
      constexpr int slot = (PH == PH_AA_ODD) ? opp(i) : i;
      constexpr int dx = shift ? -cx(i) : 0;
      constexpr int dy = shift ? -cy(i) : 0;
      gs[n][i] = ld_raw<S>(at<S>(sr[dy + 1] + slot * psb, rp[n].template of<dx>()));
    });
  }

#pragma unroll
  for (int n = 0; n < NPT; ++n) {
    T g[Q], out[Q], rv[NREC];
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = Tr::load_raw(gs[n][i]);
    collide<T, MODEL, ConserveMode<S>::value>(g, out, k, REC ? rv : nullptr);
    if constexpr (REC) {
      const RowRes rr = row_res(rec, size_t(rec_rs) * sizeof(T), y);
#pragma unroll
      for (int r = 0; r < NREC; ++r)
        stb<T, kAuxStore<WT>>(rr, r * geo.ps * int(sizeof(T)), uint32_t(rp[n].p0) * uint32_t(sizeof(T)), rv[r]);
    }
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr bool shift = (PH == PH_AA_ODD);
      constexpr int slot = (PH == PH_AA_EVEN) ? opp(i) : i;
      constexpr int dx = shift ? cx(i) : 0;
      constexpr int dy = shift ? cy(i) : 0;
      stb<S, kAuxStore<WT>>(dr[dy + 1], slot * int(psb), uint32_t(rp[n].template of<dx>()) * uint32_t(sizeof(S)),
                            Tr::store(out[i]));
    });
  }
}

// Two time steps per launch (A-B pattern), staged through LDS. A block owns kFuseGroups
// consecutive groups (one interior wavefront each) and the rows [y0, y1), the rows split
// evenly over gridDim.y row blocks (so gridDim.y <= ny); two
// halo wavefronts compute the x-neighbours of its edge groups. The block walks its rows
// y0 - 1 .. y1: phase A computes step 1 of every wavefront's node at row r from global
// memory (pull) into a ring of three rows in LDS, rounded to the storage type exactly as
// the single-step kernel would store it; phase B computes step 2 of row r - 1 for the
// interior wavefronts, pulling from the ring, and stores it. The loads of row r + 1 are
// issued before the barrier so that they overlap phase B. Every population is read once and
// written once per two steps (plus the halo's reads), and the result is bit-identical to
// two single steps: the halo nodes' step 1 is the same computation on the same inputs.
// Requires nx % 64 == 0 (no padding, so the interior x-neighbours of a group are the
// adjacent groups of the same lane) and S % kFuseGroups == 0. A block recomputes two halo
// rows of step 1 and reads four extra rows, so the host keeps blocks as tall as the grid
// allows while still giving every compute unit work, between kFuseMinRows and kFuseRows.
constexpr int kFuseGroups = 8;
constexpr int kFuseRows = 64;
constexpr int kFuseMinRows = 2;
// The FP32 pair kernels (forward, and adjoint for every storage type but FP64) also take
// blocks of up to kFuseRowsTall rows when the grid then gives each block a compute unit of its
// own. Measured on MI355X, 4096^2 (32 blocks of 128 rows against 64 of 64), us per launch on
// three machines: 217.3-218.3 / 220.1-221.0, 217.5 / 223.0, 211.2-212.4 / 215.0-215.6; the
// one-segment adjoint sweep 81.9-82.0 against 81.0-81.1 GLUPS. On 8192^2 (several rounds of
// blocks) 128-row blocks measured 1 % faster on one machine and 8.5 % slower on another
// (921-922 against 849-850 us), and the 16-bit pairs, three blocks per compute unit, 6 %
// slower: there the planner keeps kFuseRows.
constexpr int kFuseRowsTall = 128;
template <class T> struct FuseTall : std::false_type {};
template <> struct FuseTall<float> : std::true_type {};
// The hardware hands consecutive workgroup IDs to the chip's 8 XCDs in turn, and each XCD has
// its own L2. The two-step kernel renumbers its blocks so that every XCD works on one
// contiguous range of tiles, x-neighbours side by side: the halo groups a block re-reads are
// then being read at the same time by its neighbour on the same L2 (measured on MI355X:
// 38.6 instead of 45.9 B/node fetched from HBM per launch). Any value is correct (it is a
// permutation of the tiles); 8 matches MI355X.
constexpr int kXcds = 8;

// Tile (block column, row block) of the block with linear ID L = blockIdx.x + gridDim.x
// blockIdx.y: XCD L % kXcds takes tiles [start, start + count) in order, start and count
// splitting the n tiles as evenly as possible.
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int nx = int(gridDim.x), n = nx * int(gridDim.y);
  const int L = int(blockIdx.x) + int(blockIdx.y) * nx;
  const int xcd = L % kXcds;
  const int t = xcd * (n / kXcds) + min(xcd, n % kXcds) + L / kXcds;
  bx = t % nx;
  by = t / nx;
}

// Block barrier of the two-step kernels, which is also a scheduling fence: no instruction
// moves across it. Without the fence the scheduler hoisted phase A's collision (it reads only
// the registers the previous row's loads fill) above the preceding barrier and phase B, so
// each row waited for its loads before phase B instead of after it: the FP32 pair lost 5 %
// (LBGK 11 %) once its addresses no longer tied the loads to their place in the loop.
__device__ __forceinline__ void pair_sync() {
  __syncthreads();
  __builtin_amdgcn_sched_barrier(0);
}

// Whether the two-step kernel's interior wavefronts load with the nontemporal hint. Without
// it, the groups a block re-reads as halo stay in L2 for the neighbouring block that reads
// them too. Measured on MI355X, complete model, HBM bytes read per node and launch with /
// without the hint: FP64 83.0 / 73.4 (8192^2), BF16 21.8 / 19.4, FP32 38.1 / 37.0 (4096^2);
// GLUPS: FP64 76.3 -> 79.2, 16-bit unchanged (188), FP32 145.6 -> 144.4 (LBGK 155.3 ->
// 157.8). So FP32 interior wavefronts keep it; its halo wavefronts, which only load, load
// plain (140.4 -> 141.6 at 4096^2, 141.1 -> 143.1 at 8192^2, LBGK +1 %).
template <class S> struct PairLoadsNT : std::false_type {};
template <> struct PairLoadsNT<float> : std::true_type {};

template <class S, bool NT = PairLoadsNT<S>::value>
__device__ __forceinline__ void load_pulled(const S* src, const Geo& geo, int r, const RowPos& rp,
                                            typename StorageTraits<S>::Raw gs[Q]) {
  const int y = r < 0 ? r + geo.ny : (r >= geo.ny ? r - geo.ny : r);
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;
  const size_t rsb = size_t(geo.rs) * sizeof(S);
  const int psb = geo.ps * int(sizeof(S));
  const RowRes sr[3] = {row_res(src, rsb, ym), row_res(src, rsb, y), row_res(src, rsb, yp)};
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    gs[i] = ldb<S, NT>(sr[-cy(i) + 1], i * psb, uint32_t(rp.template of<-cx(i)>()) * uint32_t(sizeof(S)));
  });
}

// Storage types whose two-step kernel runs the rotated loop for its interior wavefronts
// (see k_step2). Measured on MI355X, GLUPS, complete model unless noted, same machine,
// interleaved: FP32 139.1 -> 140.8 (4096^2), 141.2 -> 142.3 (8192^2), LBGK 151.3 -> 154.4;
// FP64 75.3 -> 74.4 and BF16 / FP16 182 -> 171 (8192^2; the 16-bit kernels need 70 instead
// of 56 VGPRs with it, two blocks per compute unit instead of three), so only FP32 takes it.
template <class S> struct RotatedFuseLoop : std::false_type {};
template <> struct RotatedFuseLoop<float> : std::true_type {};

// With REC the moments of both steps are recorded (rec1: first step, rec2: second step; the
// layout and row stride rec_rs of k_step), by the interior wavefronts for the block's rows.
template <class S, int MODEL, bool REC, bool WT>
__global__ void __launch_bounds__((kFuseGroups + 2) * kLanes)
k_step2(const S* __restrict__ src, S* __restrict__ dst, Geo geo, Coef<typename StorageTraits<S>::T> k,
        typename StorageTraits<S>::T* __restrict__ rec1, typename StorageTraits<S>::T* __restrict__ rec2,
        int64_t rec_rs) {
  using T = typename StorageTraits<S>::T;
  using Tr = StorageTraits<S>;
  constexpr int G = kFuseGroups;
  __shared__ S ring[3][G + 2][Q][kLanes];
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kLanes));
  const int lane = int(threadIdx.x % kLanes);
  int bx, by;
  xcd_tile(bx, by);
  const int s0 = bx * G;
  const int y0 = int(int64_t(by) * geo.ny / gridDim.y);
  const int y1 = int(int64_t(by + 1) * geo.ny / gridDim.y);
  // Phase-A node: the wavefront's own group (w = 1..G) or the x-neighbour of an edge group.
  RowPos ra;
  if (w == 0 || w == G + 1) {
    RowPos e;
    node_pos(geo, w == 0 ? s0 : s0 + G - 1, lane, e);
    const int p = w == 0 ? e.pm : e.pp;
    node_pos(geo, p / kLanes, p % kLanes, ra);
  } else {
    node_pos(geo, s0 + w - 1, lane, ra);
  }
  const bool interior = w >= 1 && w <= G;
  const int pb = (s0 + w - 1) * kLanes + lane;  // phase-B output position
  const size_t rsb = size_t(geo.rs) * sizeof(S);
  const int psb = geo.ps * int(sizeof(S));

  typename Tr::Raw gs[Q];
  // Phase A of row r: step 1 of the wavefront's node from gs into the ring slot of row r
  // (plus its moments for the block's own rows).
  auto phase_a_m = [&](const int r, auto mask_c) {
    constexpr int MASK = decltype(mask_c)::value;
    const int slot = (r - y0 + 1) % 3;
    T g[Q], out[Q], rv[NREC];
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = Tr::load_raw(gs[i]);
    collide<T, MODEL, ConserveMode<S>::value>(g, out, k, (REC && MASK == 0x1ff) ? rv : nullptr);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if ((MASK >> i) & 1) ring[slot][w][i][lane] = Tr::store(out[i]);
    if constexpr (REC && MASK == 0x1ff) {
      if (interior && r >= y0 && r < y1) {
        const RowRes rr = row_res(rec1, size_t(rec_rs) * sizeof(T), r);
#pragma unroll
        for (int j = 0; j < NREC; ++j) stb<T, kAuxStore<WT>>(rr, j * geo.ps * int(sizeof(T)), pb * uint32_t(sizeof(T)), rv[j]);
      }
    }
  };
  using AllPops = std::integral_constant<int, 0x1ff>;
  auto phase_a = [&](const int r) { phase_a_m(r, AllPops{}); };
  // Phase B of row yr (interior wavefronts): step 2 from the ring rows yr - 1 .. yr + 1.
  auto phase_b = [&](const int yr) {
    T g[Q], out[Q];
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      g[i] = Tr::load(ring[(yr - cy(i) - y0 + 1) % 3][w - cx(i)][i][lane]);
    });
    T rv[NREC];
    collide<T, MODEL, ConserveMode<S>::value>(g, out, k, REC ? rv : nullptr);
    if constexpr (REC) {
      const RowRes rr = row_res(rec2, size_t(rec_rs) * sizeof(T), yr);
#pragma unroll
      for (int j = 0; j < NREC; ++j) stb<T, kAuxStore<WT>>(rr, j * geo.ps * int(sizeof(T)), pb * uint32_t(sizeof(T)), rv[j]);
    }
    const RowRes dr = row_res(dst, rsb, yr);
#pragma unroll
    for (int i = 0; i < Q; ++i) stb<S, kAuxStore<WT>>(dr, i * psb, pb * uint32_t(sizeof(S)), Tr::store(out[i]));
  };
  auto load = [&](const int r) { load_pulled<S>(src, geo, r, ra, gs); };
  auto load_plain = [&](const int r) { load_pulled<S, false>(src, geo, r, ra, gs); };

  // Per row r = y0 - 1 .. y1 every wavefront runs phase A of r, issues the loads of r + 1,
  // and passes two barriers; between them the interior wavefronts run phase B of r - 1
  // (from r = y0 + 1 on). That is 2 (y1 - y0) + 4 barriers for every wavefront.
  // Plain loads here: this loop runs every wavefront of the unrotated types (whose
  // PairLoadsNT is false) and only the halo wavefronts of FP32.
  auto plain_loop = [&](auto mask_c) {
    load_plain(y0 - 1);
    for (int r = y0 - 1; r <= y1; ++r) {
      phase_a_m(r, mask_c);
      if (r < y1) load_plain(r + 1);
      pair_sync();
      if (decltype(mask_c)::value == 0x1ff && interior && r > y0) phase_b(r - 1);
      pair_sync();
    }
  };
  // Phase B reads from the left halo column only the populations that move in +x (1, 5, 8),
  // from the right one only those that move in -x (3, 6, 7), so the halo wavefronts compute
  // only those (and what conservation takes them from). The ten wavefronts of a block share
  // four SIMDs, two of which carry a halo wavefront and two interior ones: their phase A, three
  // collisions between two barriers against two on the other SIMDs, sets the pace of the row.
  // Measured on MI355X against full halo collisions (us per launch, same machine): FP32
  // 4096^2 213.2 -> 210.0, 8192^2 856 -> 845, 16384 x 4096 845 -> 834; FP16 746 -> 738, BF16
  // 698 -> 681, FP64 1715 -> 1697 (8192^2); bit-identical (see fmad).
  if (w == 0) {
    plain_loop(std::integral_constant<int, (1 << 1) | (1 << 5) | (1 << 8)>{});
    return;
  }
  if (w == G + 1) {
    plain_loop(std::integral_constant<int, (1 << 3) | (1 << 6) | (1 << 7)>{});
    return;
  }
  if (!RotatedFuseLoop<S>::value) {
    plain_loop(AllPops{});
    return;
  }
  load(y0 - 1);
  // Interior wavefronts, rotated: the same sequence, with the loop entered right after the
  // loads of the next row. Vector-memory operations complete in issue order, and on every
  // path into the loop those loads are the most recent ones; so phase A, which needs only
  // them, waits with phase B's stores (issued after them) still in flight. (In the loop
  // above, a path without stores -- halo wavefronts, the first rows -- joins one with them
  // at phase A, and the wait there covers every store as well.)
  phase_a(y0 - 1);
  load(y0);
  pair_sync();
  pair_sync();
  phase_a(y0);
  load(y0 + 1);
  pair_sync();
  pair_sync();
  phase_a(y0 + 1);
  if (y0 + 1 < y1) {
    load(y0 + 2);
    for (int r = y0 + 2; r < y1; ++r) {
      pair_sync();
      phase_b(r - 2);
      pair_sync();
      phase_a(r);
      load(r + 1);
    }
    pair_sync();
    phase_b(y1 - 2);
    pair_sync();
    phase_a(y1);
  }
  pair_sync();
  phase_b(y1 - 1);
  pair_sync();
}

// Two reverse steps per launch, staged through LDS like k_step2 (same blocks, halo
// wavefronts, XCD-aware tile order and three-row ring). Phase A computes fbar^n of every
// wavefront's node at row r from fbar^{n+1} gathered at x + c_i and the records rec_hi of
// step n; phase B computes fbar^{n-1} of row r - 1 for the interior wavefronts from the
// ring and the records rec_lo of step n - 1, and stores it. The same arithmetic as two
// k_adjoint_step launches (equal up to the compiler's choice of fused multiply-adds, which
// can differ between the two kernels: relative differences of order 1e-16 in FP64 and 1e-7
// in FP32). fbar uses the
// population layout in the compute type; requires nx % 64 == 0 and S % kFuseGroups == 0.
template <class T>
__device__ __forceinline__ void load_gathered(const T* src, const Geo& geo, int r, const RowPos& rp, T fs[Q]) {
  const int y = r < 0 ? r + geo.ny : (r >= geo.ny ? r - geo.ny : r);
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;
  const size_t rsb = size_t(geo.rs) * sizeof(T), psb = size_t(geo.ps) * sizeof(T);
  const char* sr[3] = {reinterpret_cast<const char*>(src) + ym * rsb, reinterpret_cast<const char*>(src) + y * rsb,
                       reinterpret_cast<const char*>(src) + yp * rsb};
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    fs[i] = ld1(at<T>(sr[cy(i) + 1] + i * psb, rp.template of<cx(i)>()));
  });
}

template <class T>
__device__ __forceinline__ void load_record(const T* rec, const Geo& geo, int64_t rec_rs, int r, int pos, T rv[NREC]) {
  const int y = r < 0 ? r + geo.ny : (r >= geo.ny ? r - geo.ny : r);
  const char* rrow = reinterpret_cast<const char*>(rec) + y * (size_t(rec_rs) * sizeof(T));
#pragma unroll
  for (int j = 0; j < NREC; ++j) rv[j] = ld1(at<T>(rrow + j * size_t(geo.ps) * sizeof(T), pos));
}

template <class T, int MODEL>
__global__ void __launch_bounds__((kFuseGroups + 2) * kLanes)
k_adjoint_step2(const T* __restrict__ fbar_next, T* __restrict__ fbar, Geo geo, Coef<T> k,
                const T* __restrict__ rec_hi, const T* __restrict__ rec_lo, int64_t rec_rs) {
  constexpr int G = kFuseGroups;
  __shared__ T ring[3][G + 2][Q][kLanes];
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kLanes));
  const int lane = int(threadIdx.x % kLanes);
  int bx, by;
  xcd_tile(bx, by);
  const int s0 = bx * G;
  const int y0 = int(int64_t(by) * geo.ny / gridDim.y);
  const int y1 = int(int64_t(by + 1) * geo.ny / gridDim.y);
  RowPos ra;
  if (w == 0 || w == G + 1) {
    RowPos e;
    node_pos(geo, w == 0 ? s0 : s0 + G - 1, lane, e);
    const int p = w == 0 ? e.pm : e.pp;
    node_pos(geo, p / kLanes, p % kLanes, ra);
  } else {
    node_pos(geo, s0 + w - 1, lane, ra);
  }
  const bool interior = w >= 1 && w <= G;
  const int pb = (s0 + w - 1) * kLanes + lane;
  const size_t rsb = size_t(geo.rs) * sizeof(T), psb = size_t(geo.ps) * sizeof(T);

  T fs[Q], rv[NREC], rl[NREC];
  // Phase A of row r: fbar^n of the wavefront's node (gathered fbar^{n+1} in fs, its
  // records in rv) into the ring slot of row r.
  auto phase_a = [&](const int r) {
    const int slot = (r - y0 + 1) % 3;
    T fb[Q];
    collide_vjp<T, MODEL>(fs, rv, k, fb);
#pragma unroll
    for (int i = 0; i < Q; ++i) ring[slot][w][i][lane] = fb[i];
  };
  // Phase B of row yr (interior wavefronts): fbar^{n-1} from the ring rows yr - 1 .. yr + 1
  // and the records of step n - 1 in rl, stored.
  auto phase_b = [&](const int yr) {
    T g[Q], fb[Q];
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      g[i] = ring[(yr + cy(i) - y0 + 1) % 3][w + cx(i)][i][lane];
    });
    collide_vjp<T, MODEL>(g, rl, k, fb);
    char* orow = reinterpret_cast<char*>(fbar) + yr * rsb;
#pragma unroll
    for (int i = 0; i < Q; ++i) st1(at<T>(orow + i * psb, pb), fb[i]);
  };
  auto load_a = [&](const int r) {
    load_gathered<T>(fbar_next, geo, r, ra, fs);
    load_record<T>(rec_hi, geo, rec_rs, r, ra.p0, rv);
  };
  auto load_b = [&](const int yr) { load_record<T>(rec_lo, geo, rec_rs, yr, pb, rl); };

  // Per row r = y0 - 1 .. y1 every wavefront runs phase A of r, issues the loads of r + 1
  // and passes two barriers; between them the interior wavefronts run phase B of r - 1
  // (from r = y0 + 1 on) and then issue the records phase B of r will need (r < y1). The
  // records are loaded one row ahead, after the stores: vector-memory operations complete
  // in issue order, so records loaded after the next row's prefetch would make phase B
  // wait for that prefetch as well.
  load_a(y0 - 1);
  if (!interior) {
    for (int r = y0 - 1; r <= y1; ++r) {
      phase_a(r);
      if (r < y1) load_a(r + 1);
      __syncthreads();
      __syncthreads();
    }
    return;
  }
  // Interior wavefronts: the loop is entered right after the loads of the next row, the most
  // recent operations on every path into it, so both waits in its body (phase B's records,
  // issued before those loads, and phase A's loads, issued before phase B's stores and the
  // next records) leave the later operations in flight.
  phase_a(y0 - 1);
  load_a(y0);
  __syncthreads();
  __syncthreads();
  phase_a(y0);
  load_a(y0 + 1);
  __syncthreads();
  load_b(y0);
  __syncthreads();
  phase_a(y0 + 1);
  if (y0 + 1 < y1) {
    load_a(y0 + 2);
    for (int r = y0 + 2; r < y1; ++r) {
      __syncthreads();
      phase_b(r - 2);
      load_b(r - 1);
      __syncthreads();
      phase_a(r);
      load_a(r + 1);
    }
    __syncthreads();
    phase_b(y1 - 2);
    load_b(y1 - 1);
    __syncthreads();
    phase_a(y1);
  }
  __syncthreads();
  phase_b(y1 - 1);
  __syncthreads();
}

// One A-B time step with solid columns at x = 0 and x = nx - 1 (fullway bounce-back, the
// isothermal shocktube of Sec. 5): a wall node pulls its populations like any node and,
// instead of colliding, sends each back the way it came, g*_i = g_opp(i) (exact in the
// shifted storage since w_i = w_opp(i)); fluid nodes collide as in k_step. One node per
// thread, no padding access; used only for wall runs, which are small.
template <class S, int MODEL>
__global__ void __launch_bounds__(kBlock)
k_step_walls(const S* __restrict__ src, S* __restrict__ dst, Geo geo, Coef<typename StorageTraits<S>::T> k) {
  using T = typename StorageTraits<S>::T;
  using Tr = StorageTraits<S>;
  int y, lane;
  const int s0 = first_group<1>(y, lane);
  RowPos rp;
  if (y >= geo.ny || !node_pos(geo, s0, lane, rp)) return;
  const int x = lane * geo.S + s0;
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;
  const size_t rsb = size_t(geo.rs) * sizeof(S), psb = size_t(geo.ps) * sizeof(S);
  const char* sr[3] = {reinterpret_cast<const char*>(src) + ym * rsb, reinterpret_cast<const char*>(src) + y * rsb,
                       reinterpret_cast<const char*>(src) + yp * rsb};
  T g[Q], out[Q];
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    g[i] = Tr::load(ld1(at<S>(sr[-cy(i) + 1] + i * psb, rp.template of<-cx(i)>())));
  });
  if (x == 0 || x == geo.nx - 1) {
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i] = g[opp(i)];
  } else {
    collide<T, MODEL, ConserveMode<S>::value>(g, out, k, nullptr);
  }
  char* orow = reinterpret_cast<char*>(dst) + y * rsb;
#pragma unroll
  for (int i = 0; i < Q; ++i) st1(at<S>(orow + i * psb, rp.p0), Tr::store(out[i]));
}

// One reverse step of the discrete adjoint: fbar^n(x) = J(m^n(x))^T fbar*(x) with the
// reverse-streamed fbar*_i(x) = fbar^{n+1}_i(x + c_i). fbar uses the population layout in
// the compute type (geo describes it); rec holds the step's recorded moments.
template <class T, int MODEL>
__global__ void __launch_bounds__(kBlock)
k_adjoint_step(const T* __restrict__ fbar_next, T* __restrict__ fbar, Geo geo, Coef<T> k,
               const T* __restrict__ rec, int64_t rec_rs) {
  int y, lane;
  const int s0 = first_group<1>(y, lane);
  RowPos rp;
  if (y >= geo.ny || !node_pos(geo, s0, lane, rp)) return;
  const int ym = (y == 0) ? geo.ny - 1 : y - 1;
  const int yp = (y == geo.ny - 1) ? 0 : y + 1;
  const size_t rsb = size_t(geo.rs) * sizeof(T), psb = size_t(geo.ps) * sizeof(T);
  const char* nr[3] = {reinterpret_cast<const char*>(fbar_next) + ym * rsb,
                       reinterpret_cast<const char*>(fbar_next) + y * rsb,
                       reinterpret_cast<const char*>(fbar_next) + yp * rsb};
  T fs[Q];
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    fs[i] = ld1(at<T>(nr[cy(i) + 1] + i * psb, rp.of<cx(i)>()));
  });
  T rv[NREC];
  const char* rrow = reinterpret_cast<const char*>(rec) + y * (size_t(rec_rs) * sizeof(T));
#pragma unroll
  for (int r = 0; r < NREC; ++r) rv[r] = ld1(at<T>(rrow + r * psb, rp.p0));
  T fb[Q];
  collide_vjp<T, MODEL>(fs, rv, k, fb);
  char* orow = reinterpret_cast<char*>(fbar) + y * rsb;
#pragma unroll
  for (int i = 0; i < Q; ++i) st1(at<T>(orow + i * psb, rp.p0), fb[i]);
}

}  // namespace lbm
