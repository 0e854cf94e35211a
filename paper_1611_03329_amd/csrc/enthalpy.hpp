// enthalpy.hpp -- the enthalpy-based D3Q7-MRT model for solid-liquid phase
// change (Liu & He, arXiv:1611.03329, App. B, Eqs. B4-B13) in the conduction
// setting of the paper's melting test (Sec. 4.3: the velocity is zero).
//
// The stored populations are the g_k themselves (no shift).  One step per
// node: En = sum g (Eq. B7); T and f_l from En (Eqs. B8, B9); the moments of
// Eq. 36 relaxed towards n^eq = (En, 0, 0, 0, varpi c_pref T, 0, 0) (Eq. B6 at
// u = 0), the three first-order moments at the local rate zeta_alpha with
// 1/zeta_alpha = 1/2 + (alpha_l f_l + alpha_s (1 - f_l)) / csT^2 (Eq. B11,
// Sec. 4.3); g* = N^-1 n* (Eq. 43); AA-pattern streaming with the thermal wall
// rules of the temperature model (anti-bounce-back at T_w with the rest-state
// weight varpi c_pref / 6, bounce-back at adiabatic walls, periodic wrap).
#pragma once

#include "kernels.hpp"

namespace lbm {

template <class C>
struct EnthalpyConsts {
  C varpi_cpref;        // varpi c_pref (Eqs. B6, B12)
  C inv_sig_s_cpl;      // 1 / (sigma_s c_pl)
  C inv_sig_l_cpl;      // 1 / (sigma_l c_pl)
  C En_s, En_l;         // enthalpies at the solidus and the liquidus (Eq. B8)
  C inv_dEn;            // 1 / (En_l - En_s), 0 when they coincide
  C T_s, T_l;
  C alpha_l, alpha_s;   // diffusivity of each phase
  C inv_csT2;           // 3 / varpi
  C zeta_e, zeta_nu;    // rates of moments 4 and 5, 6 (Eq. 38)
};

// Eqs. B8 and B9.
template <class C>
__device__ __forceinline__ void phase_of(const EnthalpyConsts<C>& ec, C En, C& T, C& fl) {
  const C Ts = En * ec.inv_sig_s_cpl;
  const C Tl = ec.T_l + (En - ec.En_l) * ec.inv_sig_l_cpl;
  const C s = (En - ec.En_s) * ec.inv_dEn;
  const C Tm = ec.T_s + s * (ec.T_l - ec.T_s);
  const bool solid = En <= ec.En_s, liquid = En >= ec.En_l;
  T = solid ? Ts : (liquid ? Tl : Tm);
  fl = solid ? C(0) : (liquid ? C(1) : s);
}

template <class C>
__device__ __forceinline__ void collide_enthalpy(const EnthalpyConsts<C>& ec, C (&g)[7]) {
  C En = g[0];
#pragma unroll
  for (int k = 1; k < 7; ++k) En += g[k];
  C T, fl;
  phase_of<C>(ec, En, T, fl);
  const C alpha = ec.alpha_l * fl + ec.alpha_s * (C(1) - fl);
  const C za = C(1) / (C(0.5) + alpha * ec.inv_csT2);
  C d[7];
  d[0] = C(0);
  static_for<1, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    C m = C(0);
    static_for<0, 7>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int c = D3Q7::N(k, i);
      if constexpr (c == 1) m += g[i];
      else if constexpr (c == -1) m -= g[i];
      else if constexpr (c != 0) m += C(c) * g[i];
    });
    if constexpr (k <= 3) d[k] = -za * m * C(1.0 / 6.0);
    else if constexpr (k == 4) d[k] = -ec.zeta_e * (m - ec.varpi_cpref * T) * C(1.0 / 6.0);
    else d[k] = -ec.zeta_nu * m * C(1.0 / 6.0);
  });
  static_for<0, 7>([&](auto I) {
    constexpr int i = decltype(I)::value;
    C acc = g[i];
    static_for<1, 7>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr int c = D3Q7::Ninv6[i][k];
      if constexpr (c == 1) acc += d[k];
      else if constexpr (c == -1) acc -= d[k];
      else if constexpr (c != 0) acc += C(c) * d[k];
    });
    g[i] = acc;
  });
}

// Pre-collision populations of node n at parity ODD (the temperature half of
// gather with the static thermal wall rules).  g_0 sits in the second rest plane.
template <bool ODD, class S, class C>
__device__ __forceinline__ void gather_g(const KParams<C>& kp, const S& sto, int n, const Nbr& nb, C (&g)[7]) {
  g[0] = ld_g0<S, C>(sto, (uint32_t)n);
  static_for<1, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if constexpr (!ODD) {
      g[k] = ld_mg<S, C>(sto, gslot(k, (uint32_t)n));
    } else {
      constexpr int ko = D3Q7::opp(k);
      int off;
      bool in;
      link<D3Q7::e(0, k), D3Q7::e(1, k), D3Q7::e(2, k), -1>(nb, off, in);
      const uint32_t e = in ? gslot(ko, (uint32_t)(n + off)) : gslot(k, (uint32_t)n);
      C v = ld_mg<S, C>(sto, e);
      constexpr int fc = d3q7_face<k, -1>();
      g[k] = in ? v : kp.heat_a[fc] * v + kp.heat_b[fc];
    }
  });
}

template <bool ODD, class S, class C>
__device__ __forceinline__ void scatter_g(const KParams<C>& kp, const S& sto, int n, const Nbr& nb, const C (&g)[7]) {
  st_g0<S, C>(sto, (uint32_t)n, g[0]);
  static_for<1, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int ko = D3Q7::opp(k);
    if constexpr (!ODD) {
      st_mg<S, C>(sto, gslot(ko, (uint32_t)n), g[k]);
    } else {
      int off;
      bool in;
      link<D3Q7::e(0, k), D3Q7::e(1, k), D3Q7::e(2, k), +1>(nb, off, in);
      constexpr int fc = d3q7_face<k, +1>();
      const C v = in ? g[k] : kp.heat_a[fc] * g[k] + kp.heat_b[fc];
      const uint32_t e = in ? gslot(k, (uint32_t)(n + off)) : gslot(ko, (uint32_t)n);
      st_mg<S, C>(sto, e, v);
    }
  });
}

template <class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_step_enthalpy(const KParams<C> kp, const EnthalpyConsts<C> ec,
                                                             const S sto) {
  // odd steps take the blocks in reverse order: they start on the nodes the
  // even step wrote last, which the last-level cache still holds
  const int blk = ODD ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
  const int n = blk * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  int x, y, z;
  node_coords(kp, n, x, y, z);
  const Nbr nb = make_nbr(kp, x, y, z);
  C g[7];
  // FP64: loads issued at raised wavefront priority (1.6 % faster; FP32 unchanged)
  if constexpr (std::is_same<C, double>::value) __builtin_amdgcn_s_setprio(1);
  gather_g<ODD, S, C>(kp, sto, n, nb, g);
  if constexpr (std::is_same<C, double>::value) __builtin_amdgcn_s_setprio(0);
  collide_enthalpy<C>(ec, g);
  scatter_g<ODD, S, C>(kp, sto, n, nb, g);
}

// Uniform initial state g = g^eq(En0, T0) of Eq. B12 at u = 0, even layout.
template <class S, class C>
__global__ void __launch_bounds__(kMaxBlock) k_init_enthalpy(const KParams<C> kp, const S sto, double g0, double gk) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  st_g0<S, C>(sto, (uint32_t)n, C(g0));
#pragma unroll
  for (int k = 1; k < 7; ++k) st_mg<S, C>(sto, gslot(k, (uint32_t)n), C(gk));
}

// T, En and f_l of the pre-collision state (any output may be null).
template <class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_fields_enthalpy(const KParams<C> kp, const EnthalpyConsts<C> ec,
                                                               const S sto, double* T, double* En, double* fl) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  int x, y, z;
  node_coords(kp, n, x, y, z);
  const Nbr nb = make_nbr(kp, x, y, z);
  C g[7];
  gather_g<ODD, S, C>(kp, sto, n, nb, g);
  C e = g[0];
#pragma unroll
  for (int k = 1; k < 7; ++k) e += g[k];
  C t, f;
  phase_of<C>(ec, e, t, f);
  if (T) T[n] = (double)t;
  if (En) En[n] = (double)e;
  if (fl) fl[n] = (double)f;
}

template <class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_get_g(const KParams<C> kp, const S sto, double* g_out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  int x, y, z;
  node_coords(kp, n, x, y, z);
  const Nbr nb = make_nbr(kp, x, y, z);
  C g[7];
  gather_g<ODD, S, C>(kp, sto, n, nb, g);
#pragma unroll
  for (int k = 0; k < 7; ++k) g_out[(size_t)k * kp.n + n] = (double)g[k];
}

template <class S, class C>
__global__ void __launch_bounds__(kMaxBlock) k_set_g(const KParams<C> kp, const S sto, const double* g_in) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  st_g0<S, C>(sto, (uint32_t)n, C(g_in[n]));
#pragma unroll
  for (int k = 1; k < 7; ++k) st_mg<S, C>(sto, gslot(k, (uint32_t)n), C(g_in[(size_t)k * kp.n + n]));
}

}  // namespace lbm
