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
template <class S> struct StorageTraits;
template <> struct StorageTraits<double> {
  using T = double;
  static __device__ __forceinline__ double load(double v) { return v; }
  static __device__ __forceinline__ double store(double v) { return v; }
};
template <> struct StorageTraits<float> {
  using T = float;
  static __device__ __forceinline__ float load(float v) { return v; }
  static __device__ __forceinline__ float store(float v) { return v; }
};
template <> struct StorageTraits<_Float16> {
  using T = float;
  static __device__ __forceinline__ float load(_Float16 v) { return float(v); }
  static __device__ __forceinline__ _Float16 store(float v) { return _Float16(v); }
};
// bfloat16 as its raw 16 bits; stores convert with the hardware FP32 -> BF16 conversion
// (round to nearest even).
struct bf16_t { uint16_t bits; };
template <> struct StorageTraits<bf16_t> {
  using T = float;
  static __device__ __forceinline__ float load(bf16_t v) { return __uint_as_float(uint32_t(v.bits) << 16); }
  static __device__ __forceinline__ bf16_t store(float v) {
    const __bf16 h = static_cast<__bf16>(v);
    bf16_t r;
    __builtin_memcpy(&r.bits, &h, sizeof(r.bits));
    return r;
  }
};

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

// 1/x: FP32 uses the hardware reciprocal refined by one Newton step (within one ulp of the
// correctly rounded quotient); FP64 divides.
template <class T>
__device__ __forceinline__ T recip(T x) { return T(1) / x; }
template <>
__device__ __forceinline__ float recip<float>(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// ---------------------------------------------------------------------------------------
// Collision of one node on shifted populations: g -> g* (eq:lbe, first line, with the
// non-equilibrium part of the chosen model). Optionally returns the recorded moments.
//
// The arithmetic is arranged for few vector instructions (the 16-bit storage paths are
// ALU-bound): the moments come from pair sums; the equilibrium and f^OReg share the
// product Phi_x Phi_y, g*_i = P_i (drho + t_i) + E_i + Psi_i; and the moments of f^OReg that
// the corrections need (psi and the prefactor's sum) use their closed forms in N_xx and u,
// which follow from the per-axis moments of Phi: sum Phi = 1, sum c Phi = u,
// sum c^2 Phi = theta + u^2, and c^3 = c, c^4 = c^2 on {-1, 0, 1}.
template <class T, int MODEL>
__device__ __forceinline__ void collide(const T g[Q], T out[Q], const Coef<T>& k, T rec[NREC]) {
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
  const T hux = T(0.5) * ux, huy = T(0.5) * uy, hux2 = T(0.5) * ux2, huy2 = T(0.5) * uy2;
  const T dx0 = -ux2, dxp = hux2 + hux, dxm = hux2 - hux;
  const T dy0 = -uy2, dyp = huy2 + huy, dym = huy2 - huy;
  const T hx0 = k.r0 + dx0, hxp = k.r1 + dxp, hxm = k.r1 + dxm;
  const T hy0 = k.r0 + dy0, hyp = k.r1 + dyp, hym = k.r1 + dym;
  // f_i^eq - w_i rho0 = drho P_i + E_i with P_i = Phi_x Phi_y and
  // E_i = rho0 (d_x Phi_y + r_x d_y), free of cancellation against w_i rho0.
  const T rdx0 = k.rho0 * dx0, rdxp = k.rho0 * dxp, rdxm = k.rho0 * dxm;
  const T a0m = k.rr0 * dym, a00 = k.rr0 * dy0, a0p = k.rr0 * dyp;  // rho0 r_x d_y, c_x = 0
  const T a1m = k.rr1 * dym, a10 = k.rr1 * dy0, a1p = k.rr1 * dyp;  // rho0 r_x d_y, c_x = +-1
  T P[Q], E[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T hx = sel(cx(i), hxm, hx0, hxp), hy = sel(cy(i), hym, hy0, hyp);
    const T rdy = cx(i) == 0 ? sel(cy(i), a0m, a00, a0p) : sel(cy(i), a1m, a10, a1p);
    P[i] = hx * hy;
    E[i] = sel(cx(i), rdxm, rdx0, rdxp) * hy + rdy;
  }
  if (rec) {
    rec[0] = rho;
    rec[1] = ux;
    rec[2] = uy;
  }

  if (MODEL == M_BGK) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T feqs = drho * P[i] + E[i];
      out[i] = feqs + k.omb * (g[i] - feqs);
    }
    if (rec) rec[3] = rec[4] = T(0);
    return;
  }

  // Traceless non-equilibrium stress (inner sum of eq:oreg): N_xx = (D - rho(ux^2 - uy^2))/2,
  // N_xy = Pxy - rho ux uy.
  const T Dm = s13 - s24;
  const T Pxy = s57 - s68;
  const T du2 = ux2 - uy2;
  const T Nxx = T(0.5) * (Dm - rho * du2);
  const T Nxy = Pxy - jx * uy;
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
  const T Cxm = T(-1) - ux, Cx0 = -ux, Cxp = T(1) - ux;
  const T Cym = T(-1) - uy, Cy0 = -uy, Cyp = T(1) - uy;
  const T X1m = Cxm * Cxm * n1 + drho, X10 = ux2 * n1 + drho, X1p = Cxp * Cxp * n1 + drho;
  const T Y1m = Cym * Cym * n1, Y10 = uy2 * n1, Y1p = Cyp * Cyp * n1;
  const T Y2m = Cym * n2, Y20 = Cy0 * n2, Y2p = Cyp * n2;

  T Psi[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) Psi[i] = T(0);
  if (MODEL == M_PARTIAL || MODEL == M_COMPLETE) {
    // psi = sum_i c_i f_i^OReg (eq:oreg-mom-compatibility) in closed form:
    // psi_x = n1 u_x (1 - 3 theta - u_x^2), psi_y = -n1 u_y (1 - 3 theta - u_y^2).
    // Every Psi_i takes half of a psi or Pi~ component, so halves are formed directly.
    const T hpsx = n1 * hux * (k.c3 - ux2);
    const T hpsy = -(n1 * huy * (k.c3 - uy2));
    if (MODEL == M_PARTIAL) {
      // eq:partial-corrections
      Psi[1] = -hpsx;
      Psi[3] = hpsx;
      Psi[2] = -hpsy;
      Psi[4] = hpsy;
    } else {
      // Prefactor (eq:geq-prefactor-evaluation), pf = -(1/(4 theta^2)) sum (cx^2 - cy^2) f^OReg
      // with sum (cx^2 - cy^2) f^OReg = n1 (2 theta (1 - theta) + e_x + e_y),
      // e = u^2 (u^2 - 1), and the stress error's three cases (halved).
      const T exx = ux2 * (ux2 - T(1)), eyy = uy2 * (uy2 - T(1));
      const T hpf = -k.inv8th2 * (n1 * (k.b0 + (exx + eyy)));
      const T hPtxx = -hpf * (k.a0 + exx), hPtyy = hpf * (k.a0 + eyy), hPtxy = hpf * (ux * uy * du2);
      // eq:complete-corrections
      Psi[1] = hPtyy - hpsx;
      Psi[3] = hPtyy + hpsx;
      Psi[2] = hPtxx - hpsy;
      Psi[4] = hPtxx + hpsy;
      const T s = T(-0.5) * (hPtxx + hPtyy);
      Psi[5] = Psi[7] = s - T(0.5) * hPtxy;
      Psi[6] = Psi[8] = s + T(0.5) * hPtxy;
    }
  }
  // g*_i = (f_i^eq - w_i rho0) + (1 - 1/tau)(f_i^OReg + Psi_i) = P_i (drho + t_i) + E_i + Psi_i
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T u = sel(cx(i), X1m, X10, X1p) - sel(cy(i), Y1m, Y10, Y1p) +
                sel(cx(i), Cxm, Cx0, Cxp) * sel(cy(i), Y2m, Y20, Y2p);
    out[i] = P[i] * u + (E[i] + Psi[i]);
  }
}

// ---------------------------------------------------------------------------------------
// Vector-Jacobian product of one node's collision: given fbs = dJ/df* (post-collision) and the
// recorded moments (rho, ux, uy, N_xx, N_xy) of the pre-collision state, returns dJ/df.
// The post-collision populations depend on the node's populations only through
// m = (rho, j_x, j_y, D, P_xy) (and, for LBGK, directly), so dJ/df = M^T dJ/dm; dJ/dm is
// accumulated here by reverse-mode differentiation of the steps of collide().
template <class T, int MODEL>
__device__ __forceinline__ void collide_vjp(const T fbs[Q], const T rec[NREC], const Coef<T>& k, T fbar[Q]) {
  const T rho = rec[0], ux = rec[1], uy = rec[2], Nxx = rec[3], Nxy = rec[4];
  const T ux2 = ux * ux, uy2 = uy * uy;
  const T hx0 = k.r0 - ux2, hxp = k.r1 + T(0.5) * (ux2 + ux), hxm = k.r1 + T(0.5) * (ux2 - ux);
  const T hy0 = k.r0 - uy2, hyp = k.r1 + T(0.5) * (uy2 + uy), hym = k.r1 + T(0.5) * (uy2 - uy);

  T rhob = T(0), uxb = T(0), uyb = T(0), Nxxb = T(0), Nxyb = T(0);
  T hxb0 = T(0), hxbp = T(0), hxbm = T(0), hyb0 = T(0), hybp = T(0), hybm = T(0);
  T feqsb[Q], Pb[Q];
  T direct[Q];

  if (MODEL == M_BGK) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      direct[i] = k.omb * fbs[i];
      feqsb[i] = (T(1) - k.omb) * fbs[i];
      Pb[i] = T(0);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      direct[i] = T(0);
      feqsb[i] = fbs[i];
    }
    // Forward recomputation of the OReg quantities.
    const T n1 = Nxx * k.inv2th2, n2 = Nxy * (T(2) * k.inv2th2);
    const T Cxm = T(-1) - ux, Cx0 = -ux, Cxp = T(1) - ux;
    const T Cym = T(-1) - uy, Cy0 = -uy, Cyp = T(1) - uy;
    const T Sxm = Cxm * Cxm, Sx0 = Cx0 * Cx0, Sxp = Cxp * Cxp;
    const T Sym = Cym * Cym, Sy0 = Cy0 * Cy0, Syp = Cyp * Cyp;
    const T X1m = Sxm * n1, X10 = Sx0 * n1, X1p = Sxp * n1;
    const T Y1m = Sym * n1, Y10 = Sy0 * n1, Y1p = Syp * n1;
    const T Y2m = Cym * n2, Y20 = Cy0 * n2, Y2p = Cyp * n2;
    T P[Q], t[Q], fo[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      P[i] = sel(cx(i), hxm, hx0, hxp) * sel(cy(i), hym, hy0, hyp);
      t[i] = sel(cx(i), X1m, X10, X1p) - sel(cy(i), Y1m, Y10, Y1p) + sel(cx(i), Cxm, Cx0, Cxp) * sel(cy(i), Y2m, Y20, Y2p);
      fo[i] = P[i] * t[i];
    }
    // out = feqs + omb (fo + Psi)
    T fob[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) fob[i] = k.omb * fbs[i];
    if (MODEL == M_PARTIAL || MODEL == M_COMPLETE) {
      T Psib[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) Psib[i] = k.omb * fbs[i];
      const T psxb = T(0.5) * (Psib[3] - Psib[1]);
      const T psyb = T(0.5) * (Psib[4] - Psib[2]);
      if (MODEL == M_COMPLETE) {
        const T pf = -k.inv4th2 * ((fo[1] + fo[3]) - (fo[2] + fo[4]));
        const T ax = k.a0 + ux2 * (ux2 - T(1));
        const T ay = k.a0 + uy2 * (uy2 - T(1));
        const T bxy = ux * uy * (ux2 - uy2);
        const T sb = (Psib[5] + Psib[6]) + (Psib[7] + Psib[8]);
        const T Ptyyb = T(0.5) * (Psib[1] + Psib[3]) - T(0.25) * sb;
        const T Ptxxb = T(0.5) * (Psib[2] + Psib[4]) - T(0.25) * sb;
        const T Ptxyb = T(0.25) * ((Psib[6] + Psib[8]) - (Psib[5] + Psib[7]));
        const T pfb = -Ptxxb * ax + Ptyyb * ay + Ptxyb * bxy;
        const T axb = -Ptxxb * pf, ayb = Ptyyb * pf, bb = Ptxyb * pf;
        uxb += axb * (T(4) * ux2 - T(2)) * ux + bb * uy * (T(3) * ux2 - uy2);
        uyb += ayb * (T(4) * uy2 - T(2)) * uy + bb * ux * (ux2 - T(3) * uy2);
        const T q = k.inv4th2 * pfb;
        fob[1] -= q;
        fob[3] -= q;
        fob[2] += q;
        fob[4] += q;
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) fob[i] += T(cx(i)) * psxb + T(cy(i)) * psyb;
    }
    // fo_i = P_i t_i
    T X1bm = T(0), X1b0 = T(0), X1bp = T(0), Y1bm = T(0), Y1b0 = T(0), Y1bp = T(0);
    T Y2bm = T(0), Y2b0 = T(0), Y2bp = T(0), Cxbm = T(0), Cxb0 = T(0), Cxbp = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      Pb[i] = fob[i] * t[i];
      const T tb = fob[i] * P[i];
      const T cxv = sel(cx(i), Cxm, Cx0, Cxp), y2v = sel(cy(i), Y2m, Y20, Y2p);
      if (cx(i) < 0) { X1bm += tb; Cxbm += tb * y2v; } else if (cx(i) > 0) { X1bp += tb; Cxbp += tb * y2v; } else { X1b0 += tb; Cxb0 += tb * y2v; }
      if (cy(i) < 0) { Y1bm -= tb; Y2bm += tb * cxv; } else if (cy(i) > 0) { Y1bp -= tb; Y2bp += tb * cxv; } else { Y1b0 -= tb; Y2b0 += tb * cxv; }
    }
    const T n1b = (X1bm * Sxm + X1b0 * Sx0 + X1bp * Sxp) + (Y1bm * Sym + Y1b0 * Sy0 + Y1bp * Syp);
    const T n2b = Y2bm * Cym + Y2b0 * Cy0 + Y2bp * Cyp;
    Cxbm += T(2) * Cxm * (X1bm * n1);
    Cxb0 += T(2) * Cx0 * (X1b0 * n1);
    Cxbp += T(2) * Cxp * (X1bp * n1);
    const T Cybm = Y2bm * n2 + T(2) * Cym * (Y1bm * n1);
    const T Cyb0 = Y2b0 * n2 + T(2) * Cy0 * (Y1b0 * n1);
    const T Cybp = Y2bp * n2 + T(2) * Cyp * (Y1bp * n1);
    uxb -= (Cxbm + Cxb0) + Cxbp;
    uyb -= (Cybm + Cyb0) + Cybp;
    Nxxb = n1b * k.inv2th2;
    Nxyb = n2b * (T(2) * k.inv2th2);
  }
  // feqs_i = rho P_i - w_i rho0, P_i = Phi_x Phi_y
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T hx = sel(cx(i), hxm, hx0, hxp), hy = sel(cy(i), hym, hy0, hyp);
    const T P = hx * hy;
    rhob += feqsb[i] * P;
    const T pb = (MODEL == M_BGK ? T(0) : Pb[i]) + feqsb[i] * rho;
    const T bx = pb * hy, by = pb * hx;
    if (cx(i) < 0) hxbm += bx; else if (cx(i) > 0) hxbp += bx; else hxb0 += bx;
    if (cy(i) < 0) hybm += by; else if (cy(i) > 0) hybp += by; else hyb0 += by;
  }
  uxb += hxb0 * (T(-2) * ux) + hxbp * (ux + T(0.5)) + hxbm * (ux - T(0.5));
  uyb += hyb0 * (T(-2) * uy) + hybp * (uy + T(0.5)) + hybm * (uy - T(0.5));
  // Chain (rho, u, N) -> (rho, j, D, Pxy).
  const T Db = T(0.5) * Nxxb;
  const T Pxyb = Nxyb;
  rhob += T(-0.5) * Nxxb * (ux2 - uy2) - Nxyb * ux * uy;
  uxb += -Nxxb * rho * ux - Nxyb * rho * uy;
  uyb += Nxxb * rho * uy - Nxyb * rho * ux;
  const T rinv = recip(rho);
  const T jxb = uxb * rinv, jyb = uyb * rinv;
  rhob -= (uxb * ux + uyb * uy) * rinv;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    fbar[i] = direct[i] + rhob + T(cx(i)) * jxb + T(cy(i)) * jyb + T(cx(i) * cx(i) - cy(i) * cy(i)) * Db +
              T(cx(i) * cy(i)) * Pxyb;
}

}  // namespace lbm
