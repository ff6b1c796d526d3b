// Device-side building blocks of the D2Q9 OReg-GEq lattice Boltzmann step for gfx950.
//
// Populations are stored shifted, g_i = f_i - w_i rho0, with w_i = r(c_ix) r(c_iy) the guided
// equilibrium at rest (r(0) = 1 - theta, r(+-1) = theta/2). The collision below works on the
// shifted values directly: every moment the step needs is unchanged by the shift (the
// weights carry unit mass and no momentum, and their normal-stress difference and shear
// moment vanish), and the equilibrium is formed as f_i^eq - w_i rho0 without cancellation.
//
// Notation follows the paper (arXiv 2602.21242): theta reduced temperature, tau relaxation
// time, f^eq guided equilibrium (eq:guidedEq), f^OReg (eq:oreg), psi compatibility error
// (eq:oreg-mom-compatibility), Pi~ stress error (eq:guidedEq-oreg-stress-tensor-error) with
// the prefactor of eq:geq-prefactor-evaluation, Psi corrections (eq:partial-corrections,
// eq:complete-corrections).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

constexpr int Q = 9;
enum { M_BGK = 0, M_UC = 1, M_PARTIAL = 2, M_COMPLETE = 3 };
// Step phases: A-B pull step; AA step from an even time (local); AA step from an odd time.
enum { PH_AB = 0, PH_AA_EVEN = 1, PH_AA_ODD = 2 };

// D2Q9 velocities in the paper's numbering, and the opposite direction of each.
__host__ __device__ constexpr int cx(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0; }
__host__ __device__ constexpr int cy(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0; }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5); }
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp axis");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp diag");

// Pick one of three per-axis values by lattice velocity component c in {-1, 0, 1}.
template <class T>
__device__ __forceinline__ T sel(int c, T m, T z, T p) { return c < 0 ? m : (c > 0 ? p : z); }

// ---------------------------------------------------------------------------------------
// Storage element types and conversions (round to nearest even into 16-bit types).

// x rounded to FP32 with round-to-odd: the FP32 value next to x toward zero, its last
// significand bit set when x is not representable. Rounding that to a format of at most 22
// significand bits to nearest even gives the correctly rounded value of x itself (the odd
// bit stands for everything below the FP32 grid, so no tie is created or lost): FP16 has 11,
// BF16 8. Converting through a nearest-even FP32 instead rounds twice and can land on the
// wrong neighbour when x lies within half an FP32 ulp of a 16-bit tie.
__device__ __forceinline__ float f64_to_f32_odd(double x) {
  float f = float(x);
  const double fd = double(f);
  if (fd == x) return f;
  uint32_t b = __builtin_bit_cast(uint32_t, f);
  if (__builtin_fabs(fd) > __builtin_fabs(x)) b -= 1u;  // nearest was away from zero: step back
  return __builtin_bit_cast(float, b | 1u);
}

template <class S> struct StorageTraits;
template <> struct StorageTraits<double> {
  using T = double;
  using Raw = double;
  static __device__ __forceinline__ double load(double v) { return v; }
  static __device__ __forceinline__ double load_raw(double v) { return v; }
  static __device__ __forceinline__ double store(double v) { return v; }
  static __device__ __forceinline__ double from_f64(double v) { return v; }
};
template <> struct StorageTraits<float> {
  using T = float;
  using Raw = float;
  static __device__ __forceinline__ float load(float v) { return v; }
  static __device__ __forceinline__ float load_raw(float v) { return v; }
  static __device__ __forceinline__ float store(float v) { return v; }
  static __device__ __forceinline__ float from_f64(double v) { return float(v); }
};
template <> struct StorageTraits<_Float16> {
  using T = float;
  // Loaded populations wait for their use as zero-extended 32-bit bit patterns. Kept as
  // _Float16 values, the compiler packs pairs of them into one register right after the
  // loads, which stalls on the loads there instead of at their first use (the two-step
  // kernel's loads of the next row then no longer overlap the barrier and phase B).
  using Raw = uint32_t;
  static __device__ __forceinline__ float load(_Float16 v) { return float(v); }
  static __device__ __forceinline__ float load_raw(uint32_t r) {
    return float(__builtin_bit_cast(_Float16, uint16_t(r)));
  }
  static __device__ __forceinline__ _Float16 store(float v) { return _Float16(v); }
  static __device__ __forceinline__ _Float16 from_f64(double v) { return _Float16(f64_to_f32_odd(v)); }
};
// bfloat16 as its raw 16 bits; stores convert with the hardware FP32 -> BF16 conversion
// (round to nearest even).
struct bf16_t { uint16_t bits; };
template <> struct StorageTraits<bf16_t> {
  using T = float;
  using Raw = bf16_t;
  static __device__ __forceinline__ float load(bf16_t v) { return __uint_as_float(uint32_t(v.bits) << 16); }
  static __device__ __forceinline__ float load_raw(bf16_t v) { return load(v); }
  static __device__ __forceinline__ bf16_t store(float v) {
    const __bf16 h = static_cast<__bf16>(v);
    bf16_t r;
    __builtin_memcpy(&r.bits, &h, sizeof(r.bits));
    return r;
  }
  static __device__ __forceinline__ bf16_t from_f64(double v) { return store(f64_to_f32_odd(v)); }
};

// How the collision's output keeps the node's mass and momentum (see collide and conserve):
// 0 direct form, 1 populations 0, 1, 2 from the conservation laws in the compute type (FP32
// storage), 2 the same in FP16 storage precision (FP16 storage, OReg models). FP64 rounds 2^29
// times finer than FP32 and needs neither. BF16 keeps the direct form: with the FP16 form its
// error on the 8192^2 turbulence after 5000 steps fell from 5.6e-2 to 6.4e-3, but its
// throughput from 197 to 165 GLUPS (its rounding is a conversion and a shift that no FMA
// absorbs), below FP16 with the same form, which is ten times as accurate.
template <class S> struct ConserveMode { static constexpr int value = 0; };
template <> struct ConserveMode<float> { static constexpr int value = 1; };
template <> struct ConserveMode<_Float16> { static constexpr int value = 2; };

// ---------------------------------------------------------------------------------------
// Per-run constants, computed on the host in FP64 and rounded to the compute type.
template <class T>
struct Coef {
  T rho0;
  T omb;          // 1 - 1/tau
  T omb_inv2th2;  // (1 - 1/tau)/(2 theta^2)
  T r0, r1;       // rest factors 1 - theta, theta/2, rounded so that r0 + 2 r1 == 1 exactly
  T rr0, rr1;     // rho0 r0, rho0 r1
  T inv2th2;      // 1/(2 theta^2)
  T inv4th2;      // 1/(4 theta^2)
  T inv8th2;      // 1/(8 theta^2)
  T a0;           // theta (1 - 3 theta)
  T b0;           // 2 theta (1 - theta)
  T c3;           // 1 - 3 theta
};

// Moments recorded per node and step for the adjoint: rho, u_x, u_y, N_xx, N_xy.
constexpr int NREC = 5;

// a * b + c with one rounding. The collision writes every fused product this way and turns
// the compiler's own contraction off: which of two products feeding a sum the compiler fuses
// depends on how many other uses each has, so a kernel that needs only some of the outputs
// (the two-step kernel's halo columns) rounded the ones it kept differently (LBGK: 20 % of
// the populations of a 2048 x 130 grid differed after two launches).
template <class T>
__device__ __forceinline__ T fmad(T a, T b, T c) {
  if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
}

// 1/x: FP32 uses the hardware reciprocal refined by one Newton step (within one ulp of the
// correctly rounded quotient); FP64 divides.
template <class T>
__device__ __forceinline__ T recip(T x) { return T(1) / x; }
template <>
__device__ __forceinline__ float recip<float>(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// Post-collision populations 1, 2 (with MOMENTUM) and 0 recomputed from the node's mass excess
// drho and momentum j: sum_i g*_i = drho, sum_i c_i g*_i = j.
template <class T, bool MOMENTUM>
__device__ __forceinline__ void conserve(T drho, T jx, T jy, T out[Q]) {
  const T d57 = out[5] - out[7], d68 = out[6] - out[8];
  if (MOMENTUM) {
    out[1] = jx - ((d57 - d68) - out[3]);
    out[2] = jy - ((d57 + d68) - out[4]);
  }
  out[0] = drho - (((out[1] + out[3]) + (out[2] + out[4])) + ((out[5] + out[7]) + (out[6] + out[8])));
}

// The same in FP16 storage precision (OReg models): populations 1-8 are returned as FP16 values
// (g*_0 is rounded by the store). The axis populations 1-4 are rounded first; the momentum
// (r_x, r_y) they then miss goes to the four diagonal populations, (r_x + r_y)/4 to 5,
// -(r_x + r_y)/4 to 7, (r_x - r_y)/4 to 8 and -(r_x - r_y)/4 to 6, a combination that carries
// exactly that momentum and leaves the mass, the normal-stress difference D and the shear
// moment P_xy untouched; each diagonal is rounded once with its share (one fused multiply-add
// into FP16), and g*_0 takes the mass. The stored node's momentum then carries the rounding of
// the four diagonal populations, whose values are the node's smallest (equilibrium weight
// theta^2/4 against theta (1 - theta)/2 on the axes), and its mass that of g*_0, instead of
// seven and nine roundings. Measured on the 8192^2 turbulence (complete model, max error of the
// populations against the FP64 run after 100 / 1000 / 2000 / 3000 / 5000 steps): direct form
// 4.8e-4 / 1.06e-3 / - / - / 2.04e-3; diagonals rounded first and the residual split over each
// axis' pair 4.5e-4 / 6.8e-4 / 9.4e-4 / 1.08e-3 / 1.27e-3; this 3.4e-4 / 3.9e-4 / 4.3e-4 /
// 4.7e-4 / 5.3e-4, in the same time per launch as the axis-pair split (737 us per 8192^2
// two-step launch, interleaved on one machine). Not for LBGK, which keeps every
// non-equilibrium moment and whose error is not carried by the momentum: with this its error
// after 5000 steps rose from 3.3e-3 to 3.7e-3, at 9 % of its throughput.
template <bool MOMENTUM>
__device__ __forceinline__ void conserve_fp16(float drho, float jx, float jy, float out[Q]) {
#pragma clang fp contract(off)
  auto q = [](float v) { return float(_Float16(v)); };
  if (MOMENTUM) {
#pragma unroll
    for (int i = 1; i < 5; ++i) out[i] = q(out[i]);
    const float d57 = out[5] - out[7], d68 = out[6] - out[8];
    const float rx = jx - ((out[1] - out[3]) + (d57 - d68));
    const float ry = jy - ((out[2] - out[4]) + (d57 + d68));
    const float sp = rx + ry, sm = rx - ry;
    out[5] = q(fmad(0.25f, sp, out[5]));
    out[7] = q(fmad(-0.25f, sp, out[7]));
    out[8] = q(fmad(0.25f, sm, out[8]));
    out[6] = q(fmad(-0.25f, sm, out[6]));
  } else {
#pragma unroll
    for (int i = 1; i < Q; ++i) out[i] = q(out[i]);
  }
  out[0] = drho - (((out[1] + out[3]) + (out[2] + out[4])) + ((out[5] + out[7]) + (out[6] + out[8])));
}

// ---------------------------------------------------------------------------------------
// Collision of one node on shifted populations: g -> g* (eq:lbe, first line, with the
// non-equilibrium part of the chosen model). Optionally returns the recorded moments.
//
// The arithmetic is arranged for few vector instructions: the moments come from pair sums;
// the equilibrium and f^OReg share the per-axis factors Phi_x Phi_y; and the moments of f^OReg
// that the corrections need (psi and the prefactor's sum) use their closed forms in N_xx and
// u, which follow from the per-axis moments of Phi: sum Phi = 1, sum c Phi = u,
// sum c^2 Phi = theta + u^2, and c^3 = c, c^4 = c^2 on {-1, 0, 1}. The final assembly is
// g*_i = Phi_y (K_x + Phi_x v_i) + c_i with K_x = Phi_x (drho + ...) + rho0 d_x formed once per
// value of c_x: three FMAs per population. (The longer form P_i (drho + t_i) + E_i + Psi_i,
// P_i = Phi_x Phi_y, needs about six; with the two-step kernel's buffer accesses the short form
// measured faster for every storage type on MI355X: FP32 pair 150.1 -> 153.6 GLUPS at 4096^2,
// 152.2 -> 156.8 at 8192^2, FP64 pair 77.3 -> 78.5.) Every fused product is written out with
// fmad, in the places where the compiler's own contraction had put them, with contraction off,
// so that the rounding of each output does not depend on which other outputs a caller uses.
//
// With CONSERVE = 1 the populations 0, 1 and 2 are then taken from the conservation laws the
// collision obeys (eq:density-momentum; the corrections keep them, eq:genOReg-constraints):
// the post-collision mass and momentum equal the pre-collision drho and j, so
// g*_1 = j_x - (g*_5 - g*_7 - g*_6 + g*_8 - g*_3), g*_2 = j_y - (g*_5 - g*_7 + g*_6 - g*_8 - g*_4)
// and g*_0 = drho - sum_{i > 0} g*_i, which equal the values above in exact arithmetic. Rounded
// to FP32, the nine values of the direct form do not sum to drho and j exactly, and the excess
// is a smooth function of the node's state: wherever the flow is nearly uniform over large
// regions it has the same sign at every node and every step, and mass and momentum drift
// linearly. On the 16384 x 4096 double shear layer (bands at u_x = +-0.2) the FP32 run gained
// 1e-6 of its mass and 2e-5 of its kinetic energy in 3000 steps, and its populations drifted
// from the FP64 run's by 1.7e-5 (theta = 1/3) and 2.5e-5 (0.5) of max f; taken from the
// conservation laws, the drifts are 1e-11 and 1e-8 and the populations stay within 2.7e-6
// and 6.4e-7 (4096^2 Taylor-Green after 2000 steps: 2.1e-6 -> 1.2e-7). The uncorrected model
// does not conserve momentum (Sec. 3), so only its mass is taken this way. CONSERVE = 2 does it
// in FP16 storage precision (conserve_fp16) for the OReg models.
template <class T, int MODEL, int CONSERVE = 0>
__device__ __forceinline__ void collide(const T g[Q], T out[Q], const Coef<T>& k, T rec[NREC]) {
#pragma clang fp contract(off)
  // Moments (Sec. 1): rho = rho0 + sum g, j = sum c g, D = sum (cx^2 - cy^2) g, Pxy = sum cx cy g.
  const T s13 = g[1] + g[3], s24 = g[2] + g[4], s57 = g[5] + g[7], s68 = g[6] + g[8];
  const T d57 = g[5] - g[7], d68 = g[6] - g[8];
  const T drho = (g[0] + (s13 + s24)) + (s57 + s68);
  const T jx = (g[1] - g[3]) + (d57 - d68);
  const T jy = (g[2] - g[4]) + (d57 + d68);
  const T rho = k.rho0 + drho;
  const T rinv = recip(rho);
  const T ux = jx * rinv, uy = jy * rinv;
  const T ux2 = ux * ux, uy2 = uy * uy;

  // Guided equilibrium (eq:guidedEq) as a product of per-axis factors
  // Phi(0,u) = 1 - theta - u^2, Phi(+-1,u) = (theta + u^2 +- u)/2, written as rest value + d.
  const T hux = T(0.5) * ux, huy = T(0.5) * uy;
  const T dx0 = -ux2, dxp = fmad(T(0.5), ux2, hux), dxm = fmad(T(0.5), ux2, -hux);
  const T dy0 = -uy2, dyp = fmad(T(0.5), uy2, huy), dym = fmad(T(0.5), uy2, -huy);
  const T hx0 = fmad(-ux, ux, k.r0), hxp = k.r1 + dxp, hxm = k.r1 + dxm;
  const T hy0 = fmad(-uy, uy, k.r0), hyp = k.r1 + dyp, hym = k.r1 + dym;
  // f_i^eq - w_i rho0 = drho P_i + E_i with P_i = Phi_x Phi_y and
  // E_i = rho0 (d_x Phi_y + r_x d_y), free of cancellation against w_i rho0.
  const T rdx0 = k.rho0 * dx0, rdxp = k.rho0 * dxp, rdxm = k.rho0 * dxm;
  if (rec) {
    rec[0] = rho;
    rec[1] = ux;
    rec[2] = uy;
  }

  if (MODEL == M_BGK) {
    // f_i^eq - w_i rho0 = Phi_y (Phi_x drho + rho0 d_x) + rho0 r_x d_y
    const T a0m = k.rr0 * dym, a00 = k.rr0 * dy0, a0p = k.rr0 * dyp;  // rho0 r_x d_y, c_x = 0
    const T a1m = k.rr1 * dym, a10 = k.rr1 * dy0, a1p = k.rr1 * dyp;  // rho0 r_x d_y, c_x = +-1
    const T Km = fmad(hxm, drho, rdxm), K0 = fmad(hx0, drho, rdx0), Kp = fmad(hxp, drho, rdxp);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T hy = sel(cy(i), hym, hy0, hyp);
      const T rdy = cx(i) == 0 ? sel(cy(i), a0m, a00, a0p) : sel(cy(i), a1m, a10, a1p);
      const T feqs = fmad(hy, sel(cx(i), Km, K0, Kp), rdy);
      out[i] = fmad(k.omb, g[i] - feqs, feqs);
    }
    if constexpr (CONSERVE == 1) conserve<T, true>(drho, jx, jy, out);
    if (rec) rec[3] = rec[4] = T(0);
    return;
  }

  // Traceless non-equilibrium stress (inner sum of eq:oreg): N_xx = (D - rho(ux^2 - uy^2))/2,
  // N_xy = Pxy - rho ux uy.
  const T Dm = s13 - s24;
  const T Pxy = s57 - s68;
  const T du2 = fmad(-uy, uy, ux2);
  const T Nxx = T(0.5) * fmad(-rho, du2, Dm);
  const T Nxy = fmad(-jx, uy, Pxy);
  if (rec) {
    rec[3] = Nxx;
    rec[4] = Nxy;
  }
  // f_i^OReg = P_i t_i, t_i = [(Cx^2 - Cy^2) N_xx + 2 Cx Cy N_xy] / (2 theta^2), C = c - u
  // (eq:oreg). Everything downstream (psi, the prefactor, Pi~, Psi) is linear in f^OReg, so
  // the relaxation factor 1 - 1/tau is folded into N here: t, psi, pf, Pi~ and Psi below are
  // all (1 - 1/tau) times the paper's quantities. drho is folded into the x-factor so that
  // P_i (drho + t_i) is one product.
  const T n1 = Nxx * k.omb_inv2th2, n2 = Nxy * (T(2) * k.omb_inv2th2);
  const T Cxm = fmad(-jx, rinv, T(-1)), Cx0 = -ux, Cxp = fmad(-jx, rinv, T(1));
  const T Cym = fmad(-jy, rinv, T(-1)), Cy0 = -uy, Cyp = fmad(-jy, rinv, T(1));
  const T X1m = fmad(Cxm * Cxm, n1, drho), X10 = fmad(ux2, n1, drho), X1p = fmad(Cxp * Cxp, n1, drho);
  const T Y1m = Cym * Cym * n1, Y10 = uy2 * n1, Y1p = Cyp * Cyp * n1;
  const T Y2m = Cym * n2, Y20 = Cy0 * n2, Y2p = Cyp * n2;

  T Psi[Q];  // -0: rho0 r_x d_y + Psi_i is then a plain product where Psi_i vanishes
#pragma unroll
  for (int i = 0; i < Q; ++i) Psi[i] = T(-0.0);
  if (MODEL == M_PARTIAL || MODEL == M_COMPLETE) {
    // psi = sum_i c_i f_i^OReg (eq:oreg-mom-compatibility) in closed form:
    // psi_x = n1 u_x (1 - 3 theta - u_x^2), psi_y = -n1 u_y (1 - 3 theta - u_y^2).
    // Every Psi_i takes half of a psi or Pi~ component, so halves are formed directly.
    const T nhx = n1 * hux, nhy = n1 * huy, cmx = fmad(-ux, ux, k.c3), cmy = fmad(-uy, uy, k.c3);
    if (MODEL == M_PARTIAL) {
      // eq:partial-corrections
      const T hpsx = nhx * cmx, hpsy = -(nhy * cmy);
      Psi[1] = -hpsx;
      Psi[3] = hpsx;
      Psi[2] = -hpsy;
      Psi[4] = hpsy;
    } else {
      // Prefactor (eq:geq-prefactor-evaluation), pf = -(1/(4 theta^2)) sum (cx^2 - cy^2) f^OReg
      // with sum (cx^2 - cy^2) f^OReg = n1 (2 theta (1 - theta) + e_x + e_y),
      // e = u^2 (u^2 - 1), and the stress error's three cases (halved).
      const T mx = fmad(ux, ux, T(-1)), my = fmad(uy, uy, T(-1)), exx = ux2 * mx;
      const T hpf = -k.inv8th2 * (n1 * (k.b0 + fmad(uy2, my, exx)));
      // hPt_xx = -mxx, hPt_yy, hPt_xy (halved stress error); hpsx = nhx cmx, hpsy = -nhy cmy
      const T txx = fmad(ux2, mx, k.a0), tyy = fmad(uy2, my, k.a0);
      const T mxx = hpf * txx, hPtyy = hpf * tyy;
      const T hPtxy = hpf * (ux * uy * du2);
      // eq:complete-corrections
      Psi[1] = fmad(-nhx, cmx, hPtyy);
      Psi[3] = fmad(nhx, cmx, hPtyy);
      Psi[2] = fmad(nhy, cmy, -mxx);
      Psi[4] = -fmad(nhy, cmy, mxx);
      const T s = T(-0.5) * fmad(hpf, tyy, -mxx);
      Psi[5] = Psi[7] = fmad(T(-0.5), hPtxy, s);
      Psi[6] = Psi[8] = fmad(T(0.5), hPtxy, s);
    }
  }
  // g*_i = (f_i^eq - w_i rho0) + (1 - 1/tau)(f_i^OReg + Psi_i)
  //      = Phi_y (K_x + Phi_x (C_x Y2 - Y1)) + (rho0 r_x d_y + Psi_i), with
  // drho + t_i = X1 - Y1 + C_x Y2 and K_x = Phi_x X1 + rho0 d_x per value of c_x.
  // Which product of K_x is fused: measured on MI355X (two-step kernel, us per launch,
  // interleaved on one machine), rho0 d_x fused is the faster choice for FP32 storage (8192^2:
  // 838-850 against 936 with Phi_x X1 fused, whose schedule there falls into a slower memory
  // access pattern; 4096^2 209-211 against 207), Phi_x X1 fused for the others (FP16 8192^2 738
  // against 763).
  T Km, K0, Kp;
  if constexpr (CONSERVE == 1) {
    Km = fmad(k.rho0, dxm, hxm * X1m), K0 = fmad(k.rho0, dx0, hx0 * X10), Kp = fmad(k.rho0, dxp, hxp * X1p);
  } else {
    Km = fmad(hxm, X1m, rdxm), K0 = fmad(hx0, X10, rdx0), Kp = fmad(hxp, X1p, rdxp);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T hx = sel(cx(i), hxm, hx0, hxp), hy = sel(cy(i), hym, hy0, hyp);
    const T rr = cx(i) == 0 ? k.rr0 : k.rr1, dy = sel(cy(i), dym, dy0, dyp);
    const T v = fmad(sel(cx(i), Cxm, Cx0, Cxp), sel(cy(i), Y2m, Y20, Y2p), -sel(cy(i), Y1m, Y10, Y1p));
    out[i] = fmad(hy, fmad(hx, v, sel(cx(i), Km, K0, Kp)), fmad(rr, dy, Psi[i]));
  }
  if constexpr (CONSERVE == 1) conserve<T, MODEL != M_UC>(drho, jx, jy, out);
  if constexpr (CONSERVE == 2) conserve_fp16<MODEL != M_UC>(drho, jx, jy, out);
}

// ---------------------------------------------------------------------------------------
// Vector-Jacobian product of one node's collision: given fbs = dJ/df* (post-collision) and the
// recorded moments (rho, ux, uy, N_xx, N_xy) of the pre-collision state, returns dJ/df.
// The post-collision populations depend on the node's populations only through
// m = (rho, j_x, j_y, D, P_xy) (and, for LBGK, directly), so dJ/df = M^T dJ/dm. With the
// populations indexed by (c_x, c_y) the equilibrium and the OReg population are sums of
// products of a function of c_x and one of c_y (eq:guidedEq, eq:oreg), so every sum over i
// of fbs_i times such a product is a 3 x 3 bilinear form x^T F y; dJ/d(rho, u, N) is a few
// of those, and the corrections Psi (linear in f^OReg through psi and the prefactor) only
// reweight F. Checked against the complex-step derivative of the literal collision.
template <class T, int MODEL>
__device__ __forceinline__ void collide_vjp(const T fbs[Q], const T rec[NREC], const Coef<T>& k, T fbar[Q]) {
  const T rho = rec[0], ux = rec[1], uy = rec[2], Nxx = rec[3], Nxy = rec[4];
  const T ux2 = ux * ux, uy2 = uy * uy;
  // Per-axis vectors over c = -1, 0, +1 (index c + 1): the GEq factors A0 = Phi(c, u_x) and
  // their u-derivatives dA0, and for the OReg population A1 = A0 C, A2 = A0 C^2 with
  // C = c - u_x, and their u_x-derivatives (dC/du_x = -1); B* likewise in y.
  T A0[3], A1[3], A2[3], dA0[3], dA1[3], dA2[3];
  T B0[3], B1[3], B2[3], dB0[3], dB1[3], dB2[3];
  A0[0] = k.r1 + T(0.5) * (ux2 - ux), A0[1] = k.r0 - ux2, A0[2] = k.r1 + T(0.5) * (ux2 + ux);
  B0[0] = k.r1 + T(0.5) * (uy2 - uy), B0[1] = k.r0 - uy2, B0[2] = k.r1 + T(0.5) * (uy2 + uy);
  dA0[0] = ux - T(0.5), dA0[1] = T(-2) * ux, dA0[2] = ux + T(0.5);
  dB0[0] = uy - T(0.5), dB0[1] = T(-2) * uy, dB0[2] = uy + T(0.5);
  // F[a][b]: the reverse-streamed adjoint populations arranged by (c_x, c_y).
  T F[3][3];
#pragma unroll
  for (int i = 0; i < Q; ++i) F[cx(i) + 1][cy(i) + 1] = fbs[i];
  auto matvec = [](const T M[3][3], const T v[3], T out[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = M[a][0] * v[0] + M[a][1] * v[1] + M[a][2] * v[2];
  };
  auto dot = [](const T x[3], const T y[3]) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
  // Terms whose coefficient is a lattice constant of 0 are left out (a product with a zero
  // constant stays in the code, since 0 * x is NaN for infinite x: 29 of the 365 vector
  // instructions of the FP32 complete model), the others are summed in the order of the full
  // sums: for finite values the complete and uncorrected models give the full sums' results
  // bit for bit; LBGK and the partial model differ within rounding (2.5e-7 in FP32), where
  // the compiler now fuses other products.

  T uxb, uyb;
  if (MODEL != M_BGK) {
    // Weights of the OReg population f^OReg_i = P_i t_i in the output: omb fbs, plus, for the
    // corrected models, the chain through Psi, which depends on f^OReg via psi = sum c f^OReg
    // and (complete model) the prefactor, a moment of f^OReg.
    T W[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) W[a][b] = k.omb * F[a][b];
    T uxc, uyc;  // the complete model's direct u-dependence of the stress error
    if (MODEL == M_PARTIAL || MODEL == M_COMPLETE) {
      // Psi bar = omb fbs; psi bar_x = (Psib_3 - Psib_1)/2, psi bar_y = (Psib_4 - Psib_2)/2.
      const T psxb = T(0.5) * (W[0][1] - W[2][1]);
      const T psyb = T(0.5) * (W[1][0] - W[1][2]);
      if (MODEL == M_COMPLETE) {
        // Prefactor from its closed form (the moment of f^OReg), stress-error weights and
        // their direct u-dependence; the prefactor's own dependence on f^OReg enters W.
        const T pf = -k.inv4th2 * (Nxx * k.inv2th2) * (k.b0 + ux2 * (ux2 - T(1)) + uy2 * (uy2 - T(1)));
        const T ax = k.a0 + ux2 * (ux2 - T(1));
        const T ay = k.a0 + uy2 * (uy2 - T(1));
        const T bxy = ux * uy * (ux2 - uy2);
        const T sb = (W[2][2] + W[0][2]) + (W[0][0] + W[2][0]);
        const T Ptyyb = T(0.5) * (W[2][1] + W[0][1]) - T(0.25) * sb;
        const T Ptxxb = T(0.5) * (W[1][2] + W[1][0]) - T(0.25) * sb;
        const T Ptxyb = T(0.25) * ((W[0][2] + W[2][0]) - (W[2][2] + W[0][0]));
        const T pfb = -Ptxxb * ax + Ptyyb * ay + Ptxyb * bxy;
        const T axb = -Ptxxb * pf, ayb = Ptyyb * pf, bb = Ptxyb * pf;
        uxc = axb * (T(4) * ux2 - T(2)) * ux + bb * uy * (T(3) * ux2 - uy2);
        uyc = ayb * (T(4) * uy2 - T(2)) * uy + bb * ux * (ux2 - T(3) * uy2);
        const T q = k.inv4th2 * pfb;
        W[2][1] -= q;  // populations 1 and 3
        W[0][1] -= q;
        W[1][2] += q;  // populations 2 and 4
        W[1][0] += q;
      }
      // W_ab += c_a psi bar_x + c_b psi bar_y with c = a - 1 (edges one term, corners the sum).
      W[2][1] += psxb;
      W[0][1] += -psxb;
      W[1][2] += psyb;
      W[1][0] += -psyb;
      W[2][2] += psxb + psyb;
      W[0][0] += -psxb - psyb;
      W[2][0] += psxb - psyb;
      W[0][2] += -psxb + psyb;
    }
    // f^OReg_ab = [(A2_a B0_b - A0_a B2_b) N_xx + 2 A1_a B1_b N_xy] / (2 theta^2).
    const T Cx[3] = {T(-1) - ux, -ux, T(1) - ux};
    const T Cy[3] = {T(-1) - uy, -uy, T(1) - uy};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      A1[c] = A0[c] * Cx[c];
      A2[c] = A1[c] * Cx[c];
      const T tx = dA0[c] * Cx[c];
      dA1[c] = tx - A0[c];
      dA2[c] = tx * Cx[c] - T(2) * A1[c];
      B1[c] = B0[c] * Cy[c];
      B2[c] = B1[c] * Cy[c];
      const T ty = dB0[c] * Cy[c];
      dB1[c] = ty - B0[c];
      dB2[c] = ty * Cy[c] - T(2) * B1[c];
    }
    T WB0[3], WB1[3], WB2[3], WdB0[3], WdB1[3], WdB2[3];
    matvec(W, B0, WB0);
    matvec(W, B1, WB1);
    matvec(W, B2, WB2);
    matvec(W, dB0, WdB0);
    matvec(W, dB1, WdB1);
    matvec(W, dB2, WdB2);
    const T kx = Nxx * k.inv2th2, ky = Nxy * (T(2) * k.inv2th2);
    const T Nxxb = k.inv2th2 * (dot(A2, WB0) - dot(A0, WB2));
    const T Nxyb = (T(2) * k.inv2th2) * dot(A1, WB1);
    const T uxo = kx * (dot(dA2, WB0) - dot(dA0, WB2)) + ky * dot(dA1, WB1);
    const T uyo = kx * (dot(A2, WdB0) - dot(A0, WdB2)) + ky * dot(A1, WdB1);
    if (MODEL == M_COMPLETE) {
      uxb = uxc + uxo;
      uyb = uyc + uyo;
    } else {
      uxb = uxo;
      uyb = uyo;
    }
    const T Db = T(0.5) * Nxxb;
    const T Pxyb = Nxyb;
    // Equilibrium part rho A0_a B0_b (shifted by a constant).
    T FB0[3], FdB0[3];
    matvec(F, B0, FB0);
    matvec(F, dB0, FdB0);
    T rhob = dot(A0, FB0);
    uxb += rho * dot(dA0, FB0);
    uyb += rho * dot(A0, FdB0);
    // Chain (rho, u, N) -> (rho, j, D, Pxy).
    rhob += T(-0.5) * Nxxb * (ux2 - uy2) - Nxyb * ux * uy;
    uxb += -Nxxb * rho * ux - Nxyb * rho * uy;
    uyb += Nxxb * rho * uy - Nxyb * rho * ux;
    const T rinv = recip(rho);
    const T jxb = uxb * rinv, jyb = uyb * rinv;
    rhob -= (uxb * ux + uyb * uy) * rinv;
    // fbar_i = rhob + c_ix jxb + c_iy jyb + (c_ix^2 - c_iy^2) Db + c_ix c_iy Pxyb, nonzero
    // terms in this order.
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T t = rhob;
      if (cx(i) != 0) t = t + (cx(i) > 0 ? jxb : -jxb);
      if (cy(i) != 0) t = t + (cy(i) > 0 ? jyb : -jyb);
      if (cx(i) * cx(i) != cy(i) * cy(i)) t = t + (cx(i) * cx(i) > cy(i) * cy(i) ? Db : -Db);
      if (cx(i) * cy(i) != 0) t = t + (cx(i) * cy(i) > 0 ? Pxyb : -Pxyb);
      fbar[i] = t;
    }
  } else {
    // LBGK: the equilibrium part rho A0_a B0_b weighted 1 - omb, and omb fbs directly.
    const T es = T(1) - k.omb;
    T FB0[3], FdB0[3];
    matvec(F, B0, FB0);
    matvec(F, dB0, FdB0);
    T rhob = es * dot(A0, FB0);
    uxb = es * rho * dot(dA0, FB0);
    uyb = es * rho * dot(A0, FdB0);
    const T rinv = recip(rho);
    const T jxb = uxb * rinv, jyb = uyb * rinv;
    rhob -= (uxb * ux + uyb * uy) * rinv;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T t = fmad(k.omb, fbs[i], rhob);
      if (cx(i) != 0) t = t + (cx(i) > 0 ? jxb : -jxb);
      if (cy(i) != 0) t = t + (cy(i) > 0 ? jyb : -jyb);
      fbar[i] = t;
    }
  }
}

}  // namespace lbm
