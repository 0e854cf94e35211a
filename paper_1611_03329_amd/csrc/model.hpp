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
// wall rules, in the compute type C.  Passed by value (kernel arguments).
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
  C s[19];          // diagonal of Lambda (Eq. 22 / 16)
  C sh[19];         // 1 - s_k / 2
  C zeta[7];        // diagonal of Q (Eq. 38)
  C inv_dT;         // 1 / delta_T, for theta in the residual
};

// ------------------------------------------------------------------ macroscopic
// rho - rho0, T, G, u and F of one node from its shifted pre-collision state.
template <class C>
struct Macro {
  C drho;      // rho - rho0 (Eq. 25)
  C jx, jy, jz;// sum_i e_i f_i
  C dsT;       // sigma (T - T_ref) = sum_k p_k (Eq. 39)
  C T;         // temperature
  C ux, uy, uz;// Eqs. 27-28
  C Fx, Fy, Fz;// Eq. 4
};

template <class Lat, class C>
__device__ __forceinline__ Macro<C> macro(const KParams<C>& kp, const C (&h)[Lat::Q], const C (&p)[7]) {
  Macro<C> M;
  C r = C(0), jx = C(0), jy = C(0), jz = C(0);
  static_for<0, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    r += h[i];
    if constexpr (Lat::e(0, i) > 0) jx += h[i];
    if constexpr (Lat::e(0, i) < 0) jx -= h[i];
    if constexpr (Lat::e(1, i) > 0) jy += h[i];
    if constexpr (Lat::e(1, i) < 0) jy -= h[i];
    if constexpr (Lat::e(2, i) > 0) jz += h[i];
    if constexpr (Lat::e(2, i) < 0) jz -= h[i];
  });
  C st = C(0);
  static_for<0, 7>([&](auto K) { st += p[decltype(K)::value]; });
  M.drho = r;
  M.jx = jx;
  M.jy = jy;
  M.jz = jz;
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
  return M;
}

// ------------------------------------------------------------------ equilibria
// m^eq(rho, u) - m^eq(rho0, 0) row k, rho0 = 1: Eq. 21 (D3Q19, beta = 3, -5.5, -0.5)
// with the conserved rows rho and rho0 u.
template <class C>
__device__ __forceinline__ C meq_shift(D3Q19, int k, const Macro<C>& M, C inv_phi) {
  const C ux = M.ux, uy = M.uy, uz = M.uz;
  const C uu = (ux * ux + uy * uy + uz * uz) * inv_phi;
  const C pxx = (C(2) * ux * ux - uy * uy - uz * uz) * inv_phi;  // 3 p_xx^eq
  const C pww = (uy * uy - uz * uz) * inv_phi;
  switch (k) {
    case 0: return M.drho;
    case 1: return C(-11) * M.drho + C(19) * uu;
    case 2: return C(3) * M.drho - C(5.5) * uu;
    case 3: return ux;
    case 4: return C(-2.0 / 3.0) * ux;
    case 5: return uy;
    case 6: return C(-2.0 / 3.0) * uy;
    case 7: return uz;
    case 8: return C(-2.0 / 3.0) * uz;
    case 9: return pxx;
    case 10: return C(-0.5) * pxx;
    case 11: return pww;
    case 12: return C(-0.5) * pww;
    case 13: return ux * uy * inv_phi;
    case 14: return uy * uz * inv_phi;
    case 15: return uz * ux * inv_phi;
    default: return C(0);
  }
}

// Eq. 15 (D3Q15, beta = 1, -5)
template <class C>
__device__ __forceinline__ C meq_shift(D3Q15, int k, const Macro<C>& M, C inv_phi) {
  const C ux = M.ux, uy = M.uy, uz = M.uz;
  const C uu = (ux * ux + uy * uy + uz * uz) * inv_phi;
  switch (k) {
    case 0: return M.drho;
    case 1: return -M.drho + uu;
    case 2: return M.drho - C(5) * uu;
    case 3: return ux;
    case 4: return C(-7.0 / 3.0) * ux;
    case 5: return uy;
    case 6: return C(-7.0 / 3.0) * uy;
    case 7: return uz;
    case 8: return C(-7.0 / 3.0) * uz;
    case 9: return (C(2) * ux * ux - uy * uy - uz * uz) * inv_phi;
    case 10: return (uy * uy - uz * uz) * inv_phi;
    case 11: return ux * uy * inv_phi;
    case 12: return uy * uz * inv_phi;
    case 13: return uz * ux * inv_phi;
    default: return C(0);
  }
}

// Forcing moments S~_k, rho0 = 1: Eq. 23 (D3Q19)
template <class C>
__device__ __forceinline__ C forcing(D3Q19, int k, const Macro<C>& M, C inv_phi) {
  const C ux = M.ux, uy = M.uy, uz = M.uz, Fx = M.Fx, Fy = M.Fy, Fz = M.Fz;
  const C uF = (ux * Fx + uy * Fy + uz * Fz) * inv_phi;
  const C dxx = (C(2) * ux * Fx - uy * Fy - uz * Fz) * inv_phi;
  const C dww = (uy * Fy - uz * Fz) * inv_phi;
  switch (k) {
    case 1: return C(38) * uF;
    case 2: return C(-11) * uF;
    case 3: return Fx;
    case 4: return C(-2.0 / 3.0) * Fx;
    case 5: return Fy;
    case 6: return C(-2.0 / 3.0) * Fy;
    case 7: return Fz;
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
  const C ux = M.ux, uy = M.uy, uz = M.uz, Fx = M.Fx, Fy = M.Fy, Fz = M.Fz;
  const C uF = (ux * Fx + uy * Fy + uz * Fz) * inv_phi;
  switch (k) {
    case 1: return C(2) * uF;
    case 2: return C(-10) * uF;
    case 3: return Fx;
    case 4: return C(-7.0 / 3.0) * Fx;
    case 5: return Fy;
    case 6: return C(-7.0 / 3.0) * Fy;
    case 7: return Fz;
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
// Row 0 has dm_0 = 0 and S~_0 = 0, so it is skipped.  Both products use the
// symmetry of the basis: with s_i = h_i + h_ibar and d_i = h_i - h_ibar for one
// direction i of each opposite pair, even rows of M see only h_0 and the s_i,
// odd rows only the d_i; on the way back h*_i and h*_ibar share the even part
// and differ in the sign of the odd part.
template <class Lat, class C>
__device__ __forceinline__ void collide_flow(const KParams<C>& kp, const Macro<C>& M, C (&h)[Lat::Q]) {
  constexpr int Q = Lat::Q;
  C sp[Q], dp[Q];  // used at pair representatives only
  static_for<1, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (is_pair_rep<Lat>(i)) {
      sp[i] = h[i] + h[Lat::opp(i)];
      dp[i] = h[i] - h[Lat::opp(i)];
    }
  });
  C d[Q];
  static_for<1, Q>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr bool even = row_is_even<Lat>(k);
    C m = C(0);
    if constexpr (even && Lat::moment(k, 0) != 0) m = C(Lat::moment(k, 0)) * h[0];
    static_for<1, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (is_pair_rep<Lat>(i)) {
        constexpr int c = Lat::moment(k, i);
        const C v = even ? sp[i] : dp[i];
        if constexpr (c == 1) m += v;
        else if constexpr (c == -1) m -= v;
        else if constexpr (c != 0) m += C(c) * v;
      }
    });
    const C dm = m - meq_shift(Lat{}, k, M, kp.inv_phi);
    const C delta = -kp.s[k] * dm + kp.sh[k] * forcing(Lat{}, k, M, kp.inv_phi);
    d[k] = delta * C(1.0 / Lat::norm2(k));
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
    d[k] = -kp.zeta[k] * (m - eq) * C(1.0 / 6.0);
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
