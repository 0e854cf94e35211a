// model.hpp -- per-node physics of the DDF-MRT porous-convection model
// (Liu & He, arXiv:1611.03329) for the gfx950 kernels.
//
// All populations are carried SHIFTED by their rest state: h_i = f_i - w_i rho0
// and p_k = g_k - omega_k sigma T_ref.  Every function below works on the shifted
// values, so the moments it forms are departures from the rest state
// (rho0 = 1, u = 0, T = T_ref).  This keeps FP32 arithmetic well conditioned;
// in exact arithmetic it is the unshifted model.
#pragma once

#include "lattice.hpp"

namespace lbm {

// Kernel parameters: geometry, derived physical constants, relaxation rates and
// wall rules, in the compute type C.  Read in place from the member table.
template <class C>
struct KParams {
  int nx, ny, nz;
  int nxy;          // nx * ny
  double inv_nx;    // 1/nx and 1/(nx*ny) rounded up: exact quotients for n < 2^31
  double inv_nxy;
  int n;            // nodes
  int pstride;      // elements between consecutive population planes
  int per[3];       // axis is periodic
  int gaxis;        // buoyancy axis
  int moving;       // some wall face has a nonzero velocity (used when GEN)
  int open_flow;    // bit f set: face f is an open outlet for f (flow)
  int open_heat;    // bit f set: face f is an outflow face for g
  int special;      // bit f set: face f moves or is open (its nodes need the general rules)
  int sep;          // the tiled element index is a sum of an x, a y and a z part (see tile_deltas)
  C u_wall[6][3];   // wall velocity per face
  C heat_a[6];      // thermal wall rule: p_in = heat_a * p_out + heat_b (1, 0 on outflow faces)
  C heat_b[6];
  C phi, inv_phi;   // porosity
  C c_darcy;        // phi nu / K        (Eq. 4)
  C c_forch;        // phi F_phi / sqrt K (Eq. 4)
  C l0, l1;         // Eq. 28
  C l0m;            // l0 - 1/2 = phi nu / (4 K), the part of l0 that carries the Darcy drag
  C gbeta;          // g beta of Eq. 5
  C accel[3];       // a of Eq. 5
  C sigma, inv_sigma, T_ref, varpi;
  C sn[19];         // s_k / |M_k|^2: diagonal of Lambda (Eq. 22 / 16) over the row norms of M
  C shn[19];        // (1 - s_k / 2) / |M_k|^2
  C zeta6[7];       // diagonal of Q (Eq. 38) over 6 (the common denominator of Eq. 43)
  C inv_dT;         // 1 / delta_T, for theta in the residual
};

// ------------------------------------------------------------------ flow moments
// The step kernels may carry the moving flow populations multiplied by a
// power of two SC (the scale of FP16 storage: the stored values are used as
// they are) and the rest population too; moments formed from them are SC times
// the true ones.  Everything that feeds back into the populations (equilibria,
// forcing) is then formed SC times larger too, from one scaled factor per
// product, so the collision costs the same as unscaled and no population is
// scaled on its way in or out.  SC = 1 elsewhere.
//
// Pair sums and differences: for the direction i of each opposite pair with
// the smaller index, s_i = h_i + h_ibar and d_i = h_i - h_ibar.  Even moment
// rows (rho, e, eps, second- and fourth-order) see only h_0 and the s_i, odd
// rows (j, q, m) only the d_i.
template <class Lat, class C>
struct Pairs {
  C h0;
  C s[Lat::Q], d[Lat::Q];  // used at pair representatives only
};

template <class Lat, class C>
__device__ __forceinline__ Pairs<Lat, C> make_pairs(const C (&h)[Lat::Q]) {
  Pairs<Lat, C> P;
  P.h0 = h[0];
  static_for<1, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (is_pair_rep<Lat>(i)) {
      P.s[i] = h[i] + h[Lat::opp(i)];
      P.d[i] = h[i] - h[Lat::opp(i)];
    }
  });
  return P;
}

// Row K of M applied to the populations (Eq. 11), from the pair sums.
template <class Lat, int K, class C>
__device__ __forceinline__ C moment(const Pairs<Lat, C>& P) {
  constexpr bool even = row_is_even<Lat>(K);
  C m = C(0);
  bool first = true;
  if constexpr (even && Lat::moment(K, 0) != 0) {
    m = Lat::moment(K, 0) == 1 ? P.h0 : C(Lat::moment(K, 0)) * P.h0;
    first = false;
  }
  static_for<1, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (is_pair_rep<Lat>(i)) {
      constexpr int c = Lat::moment(K, i);
      const C v = even ? P.s[i] : P.d[i];
      if constexpr (c != 0) {
        if (first) m = c == 1 ? v : (c == -1 ? -v : C(c) * v);
        else if constexpr (c == 1) m += v;
        else if constexpr (c == -1) m -= v;
        else m += C(c) * v;
        first = false;
      }
    }
  });
  return m;
}

// ------------------------------------------------------------------ macroscopic
// rho - rho0, T, G, u and F of one node from its shifted pre-collision state,
// and the scaled copies the collision works with.
template <class C>
struct Macro {
  C drho;        // rho - rho0 (Eq. 25)
  C sdrho;       // SC (rho - rho0)
  C dsT;         // sigma (T - T_ref) = sum_k p_k (Eq. 39)
  C T;           // temperature
  C ux, uy, uz;  // Eqs. 27-28
  C Ux, Uy, Uz;  // SC u
  C Fx, Fy, Fz;  // Eq. 4
  C SFx, SFy, SFz;  // SC F
};

// SC is the scale of the flow populations (a power of two, exact both ways).
template <class Lat, int SC, class C>
__device__ __forceinline__ Macro<C> macro(const KParams<C>& kp, const Pairs<Lat, C>& P, const C (&p)[7]) {
  constexpr C inv = C(1.0 / SC);
  Macro<C> M;
  const C sr = moment<Lat, 0>(P);
  const C jx = moment<Lat, 3>(P) * inv, jy = moment<Lat, 5>(P) * inv, jz = moment<Lat, 7>(P) * inv;
  C st = C(0);
  static_for<0, 7>([&](auto K) { st += p[decltype(K)::value]; });
  M.sdrho = sr;
  M.drho = sr * inv;
  M.dsT = st;
  M.T = kp.T_ref + st * kp.inv_sigma;
  // Eq. 5 (buoyancy along +gaxis, T0 = T_ref)
  C G[3] = {kp.accel[0], kp.accel[1], kp.accel[2]};
  const C b = kp.gbeta * (st * kp.inv_sigma);
  G[0] += kp.gaxis == 0 ? b : C(0);
  G[1] += kp.gaxis == 1 ? b : C(0);
  G[2] += kp.gaxis == 2 ? b : C(0);
  // Eqs. 27-28 (sum over all directions, rho0 = 1, dt = 1)
  const C hp = C(0.5) * kp.phi;
  const C vx = jx + hp * G[0], vy = jy + hp * G[1], vz = jz + hp * G[2];
  // u = v / D with D = l0 + sqrt(l0^2 + l1 |v|) = 1 + delta, evaluated as
  // u = v - v delta / D with delta = 2 (l0 - 1/2) + l1 |v| / D built from its
  // small parts.  D itself is close to 1: in FP32 its rounding (or that of
  // l0 ~ 1/2) would shift the drag it carries by up to 1e-4 relative, an
  // offset the weak Darcy damping then turns into a velocity error of 1e-5.
  const C vn = sqrt(vx * vx + vy * vy + vz * vz);
  const C rD = C(1) / (kp.l0 + sqrt(kp.l0 * kp.l0 + kp.l1 * vn));
  const C q = (C(2) * kp.l0m + kp.l1 * vn * rD) * rD;
  M.ux = vx - vx * q;
  M.uy = vy - vy * q;
  M.uz = vz - vz * q;
  // Eq. 4
  const C un = sqrt(M.ux * M.ux + M.uy * M.uy + M.uz * M.uz);
  const C drag = -(kp.c_darcy + kp.c_forch * un);
  M.Fx = drag * M.ux + kp.phi * G[0];
  M.Fy = drag * M.uy + kp.phi * G[1];
  M.Fz = drag * M.uz + kp.phi * G[2];
  constexpr C sc = C(SC);
  M.Ux = M.ux * sc;
  M.Uy = M.uy * sc;
  M.Uz = M.uz * sc;
  M.SFx = M.Fx * sc;
  M.SFy = M.Fy * sc;
  M.SFz = M.Fz * sc;
  return M;
}

// ------------------------------------------------------------------ equilibria
// SC (m^eq(rho, u) - m^eq(rho0, 0)) row k, rho0 = 1: Eq. 21 (D3Q19, beta = 3,
// -5.5, -0.5).  Rows 0, 3, 5, 7 (conserved) are not needed: the collision
// skips row 0 and takes the momentum rows' change from the force directly.
template <class C>
__device__ __forceinline__ C meq_shift(D3Q19, int k, const Macro<C>& M, C inv_phi) {
  const C ux = M.ux, uy = M.uy, uz = M.uz, Ux = M.Ux, Uy = M.Uy, Uz = M.Uz;
  const C uu = (Ux * ux + Uy * uy + Uz * uz) * inv_phi;
  const C pxx = (C(2) * Ux * ux - Uy * uy - Uz * uz) * inv_phi;  // 3 p_xx^eq
  const C pww = (Uy * uy - Uz * uz) * inv_phi;
  switch (k) {
    case 1: return C(-11) * M.sdrho + C(19) * uu;
    case 2: return C(3) * M.sdrho - C(5.5) * uu;
    case 4: return C(-2.0 / 3.0) * Ux;
    case 6: return C(-2.0 / 3.0) * Uy;
    case 8: return C(-2.0 / 3.0) * Uz;
    case 9: return pxx;
    case 10: return C(-0.5) * pxx;
    case 11: return pww;
    case 12: return C(-0.5) * pww;
    case 13: return Ux * uy * inv_phi;
    case 14: return Uy * uz * inv_phi;
    case 15: return Uz * ux * inv_phi;
    default: return C(0);
  }
}

// Eq. 15 (D3Q15, beta = 1, -5)
template <class C>
__device__ __forceinline__ C meq_shift(D3Q15, int k, const Macro<C>& M, C inv_phi) {
  const C ux = M.ux, uy = M.uy, uz = M.uz, Ux = M.Ux, Uy = M.Uy, Uz = M.Uz;
  const C uu = (Ux * ux + Uy * uy + Uz * uz) * inv_phi;
  switch (k) {
    case 1: return -M.sdrho + uu;
    case 2: return M.sdrho - C(5) * uu;
    case 4: return C(-7.0 / 3.0) * Ux;
    case 6: return C(-7.0 / 3.0) * Uy;
    case 8: return C(-7.0 / 3.0) * Uz;
    case 9: return (C(2) * Ux * ux - Uy * uy - Uz * uz) * inv_phi;
    case 10: return (Uy * uy - Uz * uz) * inv_phi;
    case 11: return Ux * uy * inv_phi;
    case 12: return Uy * uz * inv_phi;
    case 13: return Uz * ux * inv_phi;
    default: return C(0);
  }
}

// SC times the forcing moments S~_k, rho0 = 1: Eq. 23 (D3Q19)
template <class C>
__device__ __forceinline__ C forcing(D3Q19, int k, const Macro<C>& M, C inv_phi) {
  const C ux = M.ux, uy = M.uy, uz = M.uz, Fx = M.SFx, Fy = M.SFy, Fz = M.SFz;
  const C uF = (ux * Fx + uy * Fy + uz * Fz) * inv_phi;
  const C dxx = (C(2) * ux * Fx - uy * Fy - uz * Fz) * inv_phi;
  const C dww = (uy * Fy - uz * Fz) * inv_phi;
  switch (k) {
    case 1: return C(38) * uF;
    case 2: return C(-11) * uF;
    case 4: return C(-2.0 / 3.0) * Fx;
    case 6: return C(-2.0 / 3.0) * Fy;
    case 8: return C(-2.0 / 3.0) * Fz;
    case 9: return C(2) * dxx;
    case 10: return -dxx;
    case 11: return C(2) * dww;
    case 12: return -dww;
    case 13: return (ux * Fy + uy * Fx) * inv_phi;
    case 14: return (uy * Fz + uz * Fy) * inv_phi;
    case 15: return (ux * Fz + uz * Fx) * inv_phi;
    default: return C(0);
  }
}

// Eq. 17 (D3Q15)
template <class C>
__device__ __forceinline__ C forcing(D3Q15, int k, const Macro<C>& M, C inv_phi) {
  const C ux = M.ux, uy = M.uy, uz = M.uz, Fx = M.SFx, Fy = M.SFy, Fz = M.SFz;
  const C uF = (ux * Fx + uy * Fy + uz * Fz) * inv_phi;
  switch (k) {
    case 1: return C(2) * uF;
    case 2: return C(-10) * uF;
    case 4: return C(-7.0 / 3.0) * Fx;
    case 6: return C(-7.0 / 3.0) * Fy;
    case 8: return C(-7.0 / 3.0) * Fz;
    case 9: return C(2) * (C(2) * ux * Fx - uy * Fy - uz * Fz) * inv_phi;
    case 10: return C(2) * (uy * Fy - uz * Fz) * inv_phi;
    case 11: return (ux * Fy + uy * Fx) * inv_phi;
    case 12: return (uy * Fz + uz * Fy) * inv_phi;
    case 13: return (ux * Fz + uz * Fx) * inv_phi;
    default: return C(0);
  }
}

// ------------------------------------------------------------------ collisions
// Flow collision in moment space (Eq. 9), in place on the shifted populations:
//   dm_k = (M h)_k - (m^eq_k - m^eq_k(rest)),
//   delta_k = -s_k dm_k + (1 - s_k/2) S~_k,
//   h*_i = h_i + sum_k M_ki delta_k / |M_k|^2          (M^-1 = M^T diag(1/|M_k|^2)).
// Row 0 has dm_0 = 0 and S~_0 = 0, so it is skipped.  The momentum rows 3, 5, 7
// need no moment either: their equilibrium is rho0 u and the closure of Eqs.
// 26-28 makes rho0 u = j + F/2, so delta = -s_j (-F/2) + (1 - s_j/2) F = F for
// every s_j (the momentum gains rho0 F per step).  The other moments come from
// the pair sums P (make_pairs); on the way back h*_i and h*_ibar share the
// even part of the update and differ in the sign of the odd part.
template <class Lat, class C>
__device__ __forceinline__ void collide_flow(const KParams<C>& kp, const Macro<C>& M, const Pairs<Lat, C>& P,
                                             C (&h)[Lat::Q]) {
  constexpr int Q = Lat::Q;
  C d[Q];
  static_for<1, Q>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if constexpr (k == 3) {
      d[k] = M.SFx * C(1.0 / Lat::norm2(k));
    } else if constexpr (k == 5) {
      d[k] = M.SFy * C(1.0 / Lat::norm2(k));
    } else if constexpr (k == 7) {
      d[k] = M.SFz * C(1.0 / Lat::norm2(k));
    } else {
      const C dm = moment<Lat, k>(P) - meq_shift(Lat{}, k, M, kp.inv_phi);
      d[k] = kp.shn[k] * forcing(Lat{}, k, M, kp.inv_phi) - kp.sn[k] * dm;
    }
  });
  // rest population: even rows only
  {
    C acc = h[0];
    static_for<1, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr int c = Lat::moment(k, 0);
      if constexpr (row_is_even<Lat>(k) && c != 0) acc += C(c) * d[k];
    });
    h[0] = acc;
  }
  static_for<1, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (is_pair_rep<Lat>(i)) {
      C ev = C(0), od = C(0);
      static_for<1, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr int c = Lat::moment(k, i);
        if constexpr (c != 0) {
          C& acc = row_is_even<Lat>(k) ? ev : od;
          if constexpr (c == 1) acc += d[k];
          else if constexpr (c == -1) acc -= d[k];
          else acc += C(c) * d[k];
        }
      });
      constexpr int io = Lat::opp(i);
      h[io] = h[io] + (ev - od);
      h[i] = h[i] + (ev + od);
    }
  });
}

// Temperature collision in moment space (Eq. 34) with N of Eq. 36 and N^-1 of
// Eq. 43, on the shifted populations:
//   dn_0 = 0, dn_1..3 = (N p)_1..3 - T u, dn_4 = (N p)_4 - varpi sigma (T - T_ref),
//   dn_5,6 = (N p)_5,6;   p*_i = p_i - sum_k Ninv_ik zeta_k dn_k.
template <class C>
__device__ __forceinline__ void collide_heat(const KParams<C>& kp, const Macro<C>& M, C (&p)[7]) {
  C d[7];
  d[0] = C(0);
  static_for<1, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    C m = C(0);
    static_for<0, 7>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int c = D3Q7::N(k, i);
      if constexpr (c == 1) m += p[i];
      else if constexpr (c == -1) m -= p[i];
      else if constexpr (c != 0) m += C(c) * p[i];
    });
    C eq = C(0);
    if constexpr (k == 1) eq = M.T * M.ux;
    if constexpr (k == 2) eq = M.T * M.uy;
    if constexpr (k == 3) eq = M.T * M.uz;
    if constexpr (k == 4) eq = kp.varpi * M.dsT;
    d[k] = -kp.zeta6[k] * (m - eq);
  });
  static_for<0, 7>([&](auto I) {
    constexpr int i = decltype(I)::value;
    C acc = p[i];
    static_for<1, 7>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr int c = D3Q7::Ninv6[i][k];
      if constexpr (c == 1) acc += d[k];
      else if constexpr (c == -1) acc -= d[k];
      else if constexpr (c != 0) acc += C(c) * d[k];
    });
    p[i] = acc;
  });
}

}  // namespace lbm
