// kernels.hpp -- gfx950 kernels of the fused DDF-MRT porous-convection step.
//
// Memory: ONE copy of the populations ("AA pattern"), population-major,
// three regions (moving f, moving g, rest f_0 and g_0), each holding its
// populations in tiles of nodes (see tiled()), node n = x + nx*(y + ny*z).
// Values are stored shifted by their rest state (see model.hpp).
//
// Time parity (streaming, Eqs. 10 and 35, done in place):
//   even step: read f_i(x) from slot i of x; collide; write f*_i(x) to slot
//              ibar of x.  After it the memory holds "swapped" post-collision
//              values.
//   odd step:  read f_i(x) = f*_i(x - e_i) from slot ibar of x - e_i (wall
//              rule if x - e_i is outside); collide; write f*_i(x) to slot i
//              of x + e_i (wall rule: into slot ibar of x if outside).  After
//              it the memory holds the natural pre-collision layout again.
// Each thread reads and writes exactly the same set of addresses, so the
// update is race-free with a single copy; every value moves through HBM once
// per step (one read and one write of 26 populations per node).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "model.hpp"

namespace lbm {

constexpr int kMaxBlock = 256;

// ------------------------------------------------------------------ storage
// Element e of the state, addressed as base + 32-bit byte offset (the host
// keeps every lattice's state below 4 GiB), which maps onto the scalar-base +
// vector-offset form of the global memory instructions.
// The state always lives in device global memory; saying so keeps the compiler
// on global (not flat) instructions also where the base pointer was itself
// loaded from memory (the batch kernel's member table).
#define LBM_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ LBM_GLOBAL T* gbl(T* p) {
  return (LBM_GLOBAL T*)p;
}
// FP16 populations are stored times 2^12 (exact both ways): departures from
// the rest state down to 1.5e-8 then lie in FP16's normal range, where it
// keeps 11 significant bits, and the largest storable departure is 16.
constexpr float kHalfScale = 4096.0f;
template <class S, class C>
__device__ __forceinline__ C ld(const S* base, uint32_t e) {
  const LBM_GLOBAL char* b = (const LBM_GLOBAL char*)base;
  const S x = *(const LBM_GLOBAL S*)(b + e * (uint32_t)sizeof(S));
  if constexpr (std::is_same<S, _Float16>::value) return static_cast<C>((float)x * (1.0f / kHalfScale));
  else return static_cast<C>(x);
}
template <class S, class C>
__device__ __forceinline__ void st(S* base, uint32_t e, C v) {
  LBM_GLOBAL char* b = (LBM_GLOBAL char*)base;
  if constexpr (std::is_same<S, _Float16>::value)
    *(LBM_GLOBAL S*)(b + e * (uint32_t)sizeof(S)) = static_cast<S>((float)v * kHalfScale);
  else
    *(LBM_GLOBAL S*)(b + e * (uint32_t)sizeof(S)) = static_cast<S>(v);
}

// The step kernels take FP16 flow populations as they are stored, times
// kHalfScale, and carry the whole flow state (the rest population too) at that
// scale through the collision (see model.hpp); no population is scaled on its
// way in or out.  Other kernels use ld / st, which convert.
template <class S>
constexpr int kFlowScale = std::is_same<typename S::MoveF, _Float16>::value ? (int)kHalfScale : 1;

template <class S, class C>
__device__ __forceinline__ C ld_raw(const S* base, uint32_t e) {
  const LBM_GLOBAL char* b = (const LBM_GLOBAL char*)base;
  const S x = *(const LBM_GLOBAL S*)(b + e * (uint32_t)sizeof(S));
  if constexpr (std::is_same<S, _Float16>::value) return static_cast<C>((float)x);
  else return static_cast<C>(x);
}

// Population storage in three regions: the moving flow populations f_1..f_{Q-1}
// (type Mf), the moving temperature populations g_1..g_6 (type Mg) and the two
// rest populations f_0, g_0 (type Rs), which never leave their node.  With FP16
// storage the flow populations are FP16, f_0 too, in a plane of its own (r0;
// the rest region then holds g_0 alone); the temperature populations stay
// FP32: the heat flux is carried by the difference of opposite g populations,
// far below FP16's resolution of each of them.
template <class Mf, class Mg, class Rs>
struct Store {
  using MoveF = Mf;
  using MoveG = Mg;
  using Rest = Rs;
  Mf* mf;
  Mg* mg;
  Rs* rs;
  Mf* r0;  // f_0 with FP16 flow storage, else unused
};

// Each region stores its populations in tiles of kTile nodes: the kTile values
// of one population for nodes [t kTile, (t + 1) kTile) are contiguous and are
// followed by the next population of the same tile, so the populations of a
// block of nodes sit together in memory instead of one plane apart each (fewer
// DRAM pages open at a time).  A region of P populations holds
// P * pstride elements, pstride a multiple of kTile.
constexpr int kTileShift = 11;
constexpr uint32_t kTile = 1u << kTileShift;
template <uint32_t P>
__device__ __forceinline__ uint32_t tiled(uint32_t pop, uint32_t n) {
  return (((n >> kTileShift) * P + pop) << kTileShift) | (n & (kTile - 1u));
}
// element of moving flow population i >= 1 and moving temperature population
// k >= 1 of node n
template <class Lat>
__device__ __forceinline__ uint32_t fslot(int i, uint32_t n) { return tiled<(uint32_t)(Lat::Q - 1)>((uint32_t)(i - 1), n); }
__device__ __forceinline__ uint32_t gslot(int k, uint32_t n) { return tiled<6u>((uint32_t)(k - 1), n); }
// The rest populations f_0 and g_0 share the rest region, tiled in pairs,
// unless the flow populations are FP16 (f_0 in r0, g_0 alone in the rest region).
template <class S>
constexpr bool kHalfRest = std::is_same<typename S::MoveF, _Float16>::value;
template <class S>
__device__ __forceinline__ uint32_t g0slot(uint32_t n) { return kHalfRest<S> ? n : tiled<2u>(1u, n); }

template <class S, class C>
__device__ __forceinline__ C ld_mf(const S& s, uint32_t e) { return ld<typename S::MoveF, C>(s.mf, e); }
// moving flow population as the step carries it: times kFlowScale<S> (RAW) or true
template <bool RAW, class S, class C>
__device__ __forceinline__ C ld_mf_as(const S& s, uint32_t e) {
  if constexpr (RAW) return ld_raw<typename S::MoveF, C>(s.mf, e);
  else return ld<typename S::MoveF, C>(s.mf, e);
}
template <class S, class C>
__device__ __forceinline__ C ld_mg(const S& s, uint32_t e) { return ld<typename S::MoveG, C>(s.mg, e); }
template <class S, class C>
__device__ __forceinline__ C ld_g0(const S& s, uint32_t n) { return ld<typename S::Rest, C>(s.rs, g0slot<S>(n)); }
// f_0 as the step carries it: times kFlowScale<S> (RAW) or true
template <bool RAW, class S, class C>
__device__ __forceinline__ C ld_f0_as(const S& s, uint32_t n) {
  if constexpr (kHalfRest<S>) return RAW ? ld_raw<_Float16, C>(s.r0, n) : ld<_Float16, C>(s.r0, n);
  else return ld<typename S::Rest, C>(s.rs, tiled<2u>(0u, n));
}
template <class S, class C>
__device__ __forceinline__ void st_mf(const S& s, uint32_t e, C v) { st<typename S::MoveF, C>(s.mf, e, v); }
template <class S, class C>
__device__ __forceinline__ void st_mg(const S& s, uint32_t e, C v) { st<typename S::MoveG, C>(s.mg, e, v); }
template <class S, class C>
__device__ __forceinline__ void st_g0(const S& s, uint32_t n, C v) { st<typename S::Rest, C>(s.rs, g0slot<S>(n), v); }
// f_0 given as true value, rounded to nearest (initial and caller-given states)
template <class S, class C>
__device__ __forceinline__ void st_f0(const S& s, uint32_t n, C v) {
  if constexpr (kHalfRest<S>) st<_Float16, C>(s.r0, n, v);
  else st<typename S::Rest, C>(s.rs, tiled<2u>(0u, n), v);
}

// FP16 flow storage rounds stochastically: a value goes to one of its two
// neighbouring FP16 numbers with probability falling linearly with the
// distance, so the rounding error has zero mean.  Rounding to nearest gives
// each steady node the same error at every step, a bias that the slow
// diffusive and Darcy modes accumulate over thousands of steps; a zero-mean
// error averages out instead.  The random bits are a hash of (step, node)
// spread over the node's populations by a Weyl sequence (scatter), so runs are
// reproducible bit for bit.
template <class S>
constexpr bool kStochastic = std::is_same<typename S::MoveF, _Float16>::value;

// C. Wellons' "lowbias32" integer hash (a bijection of 32-bit words).
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// f to FP16 with the random bits r13 (uniform in [0, 2^13)): add them to the
// magnitude bits of f below FP16's 10-bit fraction, then cut those 13 bits off,
// which leaves an FP16 number exactly for magnitudes in FP16's normal range.
// Below it (2^-14, subnormals: stored departures under 1.5e-8) the conversion
// then rounds to nearest.  Infinities and the quiet NaN the hardware produces
// (fraction 0x400000) keep their class: the carry of the added bits never
// reaches their exponent; magnitudes from 65520 up convert to infinity.
__device__ __forceinline__ _Float16 half_sr(float f, uint32_t r13) {
  const uint32_t u = __float_as_uint(f);
  return (_Float16)__uint_as_float((u + r13) & ~0x1FFFu);
}

// Store of a moving flow population given as the step carries it (RAW: times
// kFlowScale<S>; else true); with FP16 storage r13 drives the rounding.
template <bool RAW, class S, class C>
__device__ __forceinline__ void st_mf_r(const S& s, uint32_t e, C v, uint32_t r13) {
  if constexpr (kStochastic<S>) {
    LBM_GLOBAL char* b = (LBM_GLOBAL char*)s.mf;
    const float f = RAW ? (float)v : (float)v * kHalfScale;
    *(LBM_GLOBAL _Float16*)(b + e * 2u) = half_sr(f, r13);
  } else {
    (void)r13;
    st_mf<S, C>(s, e, v);
  }
}

// Store of f_0 given as the step carries it (RAW: times kFlowScale<S>; else
// true); with FP16 storage r13 drives the rounding, as for st_mf_r.
template <bool RAW, class S, class C>
__device__ __forceinline__ void st_f0_r(const S& s, uint32_t n, C v, uint32_t r13) {
  if constexpr (kHalfRest<S>) {
    LBM_GLOBAL char* b = (LBM_GLOBAL char*)s.r0;
    const float f = RAW ? (float)v : (float)v * kHalfScale;
    *(LBM_GLOBAL _Float16*)(b + n * 2u) = half_sr(f, r13);
  } else {
    (void)r13;
    st<typename S::Rest, C>(s.rs, tiled<2u>(0u, n), v);
  }
}

// ------------------------------------------------------------------ geometry
// Coordinates of node n: exact division by an FP64 reciprocal rounded up
// (kp.inv_nx, kp.inv_nxy), valid for n < 2^31.
template <class C>
__device__ __forceinline__ void node_coords(const KParams<C>& kp, int n, int& x, int& y, int& z) {
  const int yz = (int)((double)n * kp.inv_nx);
  z = (int)((double)n * kp.inv_nxy);
  x = n - yz * kp.nx;
  y = yz - z * kp.ny;
}

// Offsets (in nodes) to the neighbour at coordinate -1 / +1 along each axis,
// with periodic wrap, and whether that neighbour exists.
struct Nbr {
  int off[3][2];
  bool in[3][2];
};

template <class C>
__device__ __forceinline__ Nbr make_nbr(const KParams<C>& kp, int x, int y, int z) {
  Nbr b;
  const int c[3] = {x, y, z};
  const int dim[3] = {kp.nx, kp.ny, kp.nz};
  const int str[3] = {1, kp.nx, kp.nxy};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool lo = c[a] > 0, hi = c[a] < dim[a] - 1;
    b.in[a][0] = lo || kp.per[a];
    b.in[a][1] = hi || kp.per[a];
    b.off[a][0] = (lo ? -1 : dim[a] - 1) * str[a];
    b.off[a][1] = (hi ? 1 : -(dim[a] - 1)) * str[a];
  }
  return b;
}

// Link along velocity e taken with sign SG (+1: to x + e, -1: to x - e):
// node offset and whether the linked node exists.
// Separable tiles (kp.sep): when tiles hold whole rows and planes hold whole
// tiles (or a row holds whole tiles), the element index of moving flow
// population p at node m splits as fslot(p, m) = X(x) + Y(y) + Z(z) + (p-1)
// kTile.  A link's target index is then the node's own fslot(1, n) plus one
// delta per axis it moves along, the same for every population: six deltas
// per node replace the index arithmetic of each of the 18 (14) links.
template <class Lat>
__device__ __forceinline__ void tile_deltas(const Nbr& b, int n, uint32_t f1, int (&td)[3][2]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int s = 0; s < 2; ++s) td[a][s] = (int)(fslot<Lat>(1, (uint32_t)(n + b.off[a][s])) - f1);
}

// Index delta and existence of the link along velocity e taken with sign SG,
// from the per-axis deltas of tile_deltas.
template <int EX, int EY, int EZ, int SG>
__device__ __forceinline__ void link_delta(const Nbr& b, const int (&td)[3][2], int& dl, bool& in) {
  dl = 0;
  in = true;
  if constexpr (EX != 0) {
    constexpr int s = EX * SG > 0 ? 1 : 0;
    dl += td[0][s];
    in = in && b.in[0][s];
  }
  if constexpr (EY != 0) {
    constexpr int s = EY * SG > 0 ? 1 : 0;
    dl += td[1][s];
    in = in && b.in[1][s];
  }
  if constexpr (EZ != 0) {
    constexpr int s = EZ * SG > 0 ? 1 : 0;
    dl += td[2][s];
    in = in && b.in[2][s];
  }
}

template <int EX, int EY, int EZ, int SG>
__device__ __forceinline__ void link(const Nbr& b, int& off, bool& in) {
  off = 0;
  in = true;
  if constexpr (EX != 0) {
    constexpr int s = EX * SG > 0 ? 1 : 0;
    off += b.off[0][s];
    in = in && b.in[0][s];
  }
  if constexpr (EY != 0) {
    constexpr int s = EY * SG > 0 ? 1 : 0;
    off += b.off[1][s];
    in = in && b.in[1][s];
  }
  if constexpr (EZ != 0) {
    constexpr int s = EZ * SG > 0 ? 1 : 0;
    off += b.off[2][s];
    in = in && b.in[2][s];
  }
}

// For a link that leaves the box: the face whose rule applies (the first wall
// face crossed in face order, else the first open face crossed) and whether it
// is an open face.  Open faces are those in open_mask.
template <int EX, int EY, int EZ, int SG>
__device__ __forceinline__ int exit_face(const Nbr& b, int open_mask, bool& open) {
  int wall = -1, opn = -1;
  auto axis = [&](int a, int e) {
    if (e == 0) return;
    const int side = e * SG > 0 ? 1 : 0;
    if (!b.in[a][side]) {
      const int fc = 2 * a + side;
      if ((open_mask >> fc) & 1) {
        opn = opn < 0 ? fc : opn;
      } else {
        wall = wall < 0 ? fc : wall;
      }
    }
  };
  axis(0, EX);
  axis(1, EY);
  axis(2, EZ);
  open = wall < 0 && opn >= 0;
  return wall >= 0 ? wall : (opn >= 0 ? opn : 0);
}

// Face crossed by a D3Q7 link (one axis), known at compile time.
template <int K, int SG>
constexpr int d3q7_face() {
  constexpr int a = D3Q7::e(0, K) != 0 ? 0 : (D3Q7::e(1, K) != 0 ? 1 : 2);
  constexpr int e = D3Q7::e(a, K);
  return 2 * a + (e * SG > 0 ? 1 : 0);
}

template <class Lat, int J>
__host__ __device__ constexpr double weight() {
  if constexpr (Lat::Q == 19) return Lat::w36(J) / 36.0;
  else return Lat::w72(J) / 72.0;
}

// Open outlet at rho0: the population entering along direction j is the
// anti-bounce-back of the outgoing post-collision one to twice the even part of
// f^eq(rho0, u) (Eq. 24 / 18) at the node's own velocity; shifted:
// h_j = -h*_jbar + 2 w_j [(e_j.u)^2 / (2 phi cs^4) - u^2 / (2 phi cs^2)].
// (h_out and the result SC times the true values.)
template <class Lat, int J, int SC, class C>
__device__ __forceinline__ C open_flow_value(C h_out, const Macro<C>& M, C inv_phi) {
  constexpr int ex = Lat::e(0, J), ey = Lat::e(1, J), ez = Lat::e(2, J);
  const C eu = C(ex) * M.ux + C(ey) * M.uy + C(ez) * M.uz;
  const C uu = M.ux * M.ux + M.uy * M.uy + M.uz * M.uz;
  return -h_out + C(2.0 * SC * weight<Lat, J>()) * (C(4.5) * eu * eu - C(1.5) * uu) * inv_phi;
}

// Outflow face for g: anti-bounce-back to the node's own temperature;
// shifted: p_k = -p*_kbar + 2 omega_k sigma (T - T_ref), omega_k = varpi / 6.
template <class C>
__device__ __forceinline__ C open_heat_value(const KParams<C>& kp, C p_out, const Macro<C>& M) {
  return -p_out + C(2.0 / 6.0) * kp.varpi * M.dsT;
}

// ------------------------------------------------------------------ special faces
// Face f = 2a + s (axis a, s = 0 low, 1 high) is crossed by the link along
// velocity e taken with sign SG (+1: to x + e, -1: to x - e) when the link's
// component along a points out of that face.
template <int EX, int EY, int EZ, int SG>
constexpr bool crosses(int f) {
  const int a = f >> 1;
  const int c = (a == 0 ? EX : (a == 1 ? EY : EZ)) * SG;
  return (f & 1) ? c > 0 : c < 0;
}

// Moving-wall term of bounce-back on face f for the population entering along
// direction j: 2 w_j rho0 (e_j . u_w) / cs^2 = 6 w_j (e_j . u_w), uniform over
// the face.
template <class Lat, int J, int F, class C>
__device__ __forceinline__ C wall_term_face(const KParams<C>& kp) {
  constexpr int ex = Lat::e(0, J), ey = Lat::e(1, J), ez = Lat::e(2, J);
  return C(6.0 * weight<Lat, J>()) * (C(ex) * kp.u_wall[F][0] + C(ey) * kp.u_wall[F][1] + C(ez) * kp.u_wall[F][2]);
}

// Odd-parity gather on moving walls: the population entering node n from
// outside through a moving face takes the face's wall term.  Face by face,
// for each special face some node of the wavefront lies on, only the links
// crossing it; a link crossing several faces takes the rule of its exit face
// (exit_face: the first wall face crossed, else the first open face), and an
// open exit face brings a value that is already final.
template <class Lat, int SC, class C>
__device__ __forceinline__ void gather_walls(const KParams<C>& kp, const Nbr& nb, C (&h)[Lat::Q]) {
  if (!kp.moving) return;
  static_for<0, 6>([&](auto F) {
    constexpr int f = decltype(F)::value;
    const bool on = !nb.in[f >> 1][f & 1];
    if (((kp.special >> f) & 1) && __ballot(on) != 0) {
      static_for<1, Lat::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (crosses<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), -1>(f)) {
          bool open;
          const int fc = exit_face<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), -1>(nb, kp.open_flow, open);
          const C t = wall_term_face<Lat, i, f, C>(kp) * C(SC);
          h[i] = (on && fc == f && !open) ? h[i] + t : h[i];
        }
      });
    }
  });
}

// Scatter on special faces, after the lean scatter has stored every population
// leaving through a face into this node's own opposite slot (bounce-back): for
// each special face some node of the wavefront lies on, the populations
// leaving through it are stored again with their rule applied.  Flow: at odd
// parity the open-face value or the moving-wall term, at even parity the
// open-face value (slot ibar of this node is read back only by this node when
// i leaves through an open face).  Heat: the outflow value, at both parities.
template <class Lat, bool ODD, bool RAW, class S, class C>
__device__ __forceinline__ void scatter_faces(const KParams<C>& kp, const S& sto, int n, const Nbr& nb,
                                              const C (&h)[Lat::Q], const C (&p)[7], const Macro<C>& M,
                                              uint32_t seed) {
  constexpr int SC = RAW ? kFlowScale<S> : 1;
  static_for<0, 6>([&](auto F) {
    constexpr int f = decltype(F)::value;
    const bool on = !nb.in[f >> 1][f & 1];
    const bool flow = ODD ? ((kp.special >> f) & 1) : ((kp.open_flow >> f) & 1);
    if (flow && __ballot(on) != 0) {
      static_for<1, Lat::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (crosses<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), +1>(f)) {
          constexpr int io = Lat::opp(i);
          bool open;
          const int fc = exit_face<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), +1>(nb, kp.open_flow, open);
          if (on && fc == f && (ODD || open)) {
            const C v = open ? open_flow_value<Lat, io, SC, C>(h[i], M, kp.inv_phi)
                             : h[i] + wall_term_face<Lat, io, f, C>(kp) * C(SC);
            const uint32_t r = mix32(seed + (uint32_t)n * 0x9E3779B9u + (uint32_t)i * 0x85EBCA6Bu);
            st_mf_r<RAW, S, C>(sto, fslot<Lat>(io, (uint32_t)n), v, r >> 19);
          }
        }
      });
    }
    if (((kp.open_heat >> f) & 1) && __ballot(on) != 0) {
      static_for<1, 7>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (d3q7_face<k, +1>() == f) {
          if (on) st_mg<S, C>(sto, gslot(D3Q7::opp(k), (uint32_t)n), open_heat_value<C>(kp, p[k], M));
        }
      });
    }
  });
}

// ------------------------------------------------------------------ gather
// Pre-collision shifted populations of node n at the current parity.  At odd
// parity a population entering from outside is read from this node's own slot:
// raw for walls (then the wall rule is applied), already final for open faces
// (the step that stored it applied the open rule).  The lean rules (periodic
// faces, static walls, thermal walls) are applied link by link; GEN adds the
// rules of moving walls and open faces (special faces) as corrections, face by
// face (gather_walls, scatter_faces).  SEP takes the flow links' indices from
// tile_deltas (separable tiles only).
// RAW (the step kernels): the flow populations come out times kFlowScale<S>.
template <class Lat, bool ODD, bool GEN, class S, class C, bool SEP = false, bool RAW = false>
__device__ __forceinline__ void gather(const KParams<C>& kp, const S& sto, int n, const Nbr& nb,
                                       C (&h)[Lat::Q], C (&p)[7]) {
  constexpr int SC = RAW ? kFlowScale<S> : 1;
  h[0] = ld_f0_as<RAW, S, C>(sto, (uint32_t)n);
  const uint32_t f1 = fslot<Lat>(1, (uint32_t)n);
  int td[3][2];
  if constexpr (ODD && SEP) tile_deltas<Lat>(nb, n, f1, td);
  static_for<1, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (!ODD) {
      h[i] = ld_mf_as<RAW, S, C>(sto, fslot<Lat>(i, (uint32_t)n));
    } else if constexpr (SEP) {
      constexpr int io = Lat::opp(i);
      int dl;
      bool in;
      link_delta<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), -1>(nb, td, dl, in);
      const uint32_t e = f1 + (in ? ((uint32_t)(io - 1) << kTileShift) + (uint32_t)dl
                                  : ((uint32_t)(i - 1) << kTileShift));
      h[i] = ld_mf_as<RAW, S, C>(sto, e);
    } else {
      constexpr int io = Lat::opp(i);
      int off;
      bool in;
      link<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), -1>(nb, off, in);
      const uint32_t e = in ? fslot<Lat>(io, (uint32_t)(n + off)) : fslot<Lat>(i, (uint32_t)n);
      h[i] = ld_mf_as<RAW, S, C>(sto, e);
    }
  });
  if constexpr (GEN && ODD) gather_walls<Lat, SC, C>(kp, nb, h);
  p[0] = ld_g0<S, C>(sto, (uint32_t)n);
  static_for<1, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if constexpr (!ODD) {
      p[k] = ld_mg<S, C>(sto, gslot(k, (uint32_t)n));
    } else {
      constexpr int ko = D3Q7::opp(k);
      int off;
      bool in;
      link<D3Q7::e(0, k), D3Q7::e(1, k), D3Q7::e(2, k), -1>(nb, off, in);
      const uint32_t e = in ? gslot(ko, (uint32_t)(n + off)) : gslot(k, (uint32_t)n);
      C v = ld_mg<S, C>(sto, e);
      // outflow faces carry heat_a = 1, heat_b = 0: their value is already final
      constexpr int fc = d3q7_face<k, -1>();
      v = in ? v : kp.heat_a[fc] * v + kp.heat_b[fc];
      p[k] = v;
    }
  });
}

// ------------------------------------------------------------------ scatter
// Post-collision shifted populations of node n, written for the next parity.
// M holds the node's macroscopic state (used by the open-face rules).
// RAW (the step kernels): h comes in times kFlowScale<S>.
template <class Lat, bool ODD, bool GEN, class S, class C, bool SEP = false, bool RAW = false>
__device__ __forceinline__ void scatter(const KParams<C>& kp, const S& sto, int n, const Nbr& nb,
                                        const C (&h)[Lat::Q], const C (&p)[7], const Macro<C>& M, uint32_t seed) {
  constexpr int SC = RAW ? kFlowScale<S> : 1;
  // random bits for the stochastic FP16 rounding: one hashed word per node and
  // step, and for population i the top 13 bits of that word plus i times the
  // golden-ratio constant (a Weyl sequence): each population's bits are
  // uniform, and the node's populations take evenly spread rotations of them
  const uint32_t rnd = kStochastic<S> ? mix32(seed + (uint32_t)n) : 0u;
  st_f0_r<RAW, S, C>(sto, (uint32_t)n, h[0], rnd >> 19);
  const uint32_t f1 = fslot<Lat>(1, (uint32_t)n);
  int td[3][2];
  if constexpr (ODD && SEP) tile_deltas<Lat>(nb, n, f1, td);
  static_for<1, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int io = Lat::opp(i);
    const uint32_t r = kStochastic<S> ? (rnd + (uint32_t)i * 0x9E3779B9u) >> 19 : 0u;
    if constexpr (!ODD) {
      st_mf_r<RAW, S, C>(sto, fslot<Lat>(io, (uint32_t)n), h[i], r);
    } else if constexpr (SEP) {
      int dl;
      bool in;
      link_delta<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), +1>(nb, td, dl, in);
      const uint32_t e = f1 + (in ? ((uint32_t)(i - 1) << kTileShift) + (uint32_t)dl
                                  : ((uint32_t)(io - 1) << kTileShift));
      st_mf_r<RAW, S, C>(sto, e, h[i], r);
    } else {
      int off;
      bool in;
      link<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), +1>(nb, off, in);
      const uint32_t e = in ? fslot<Lat>(i, (uint32_t)(n + off)) : fslot<Lat>(io, (uint32_t)n);
      st_mf_r<RAW, S, C>(sto, e, h[i], r);
    }
  });
  st_g0<S, C>(sto, (uint32_t)n, p[0]);
  static_for<1, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int ko = D3Q7::opp(k);
    if constexpr (!ODD) {
      st_mg<S, C>(sto, gslot(ko, (uint32_t)n), p[k]);
    } else {
      int off;
      bool in;
      link<D3Q7::e(0, k), D3Q7::e(1, k), D3Q7::e(2, k), +1>(nb, off, in);
      constexpr int fc = d3q7_face<k, +1>();
      const C v = in ? p[k] : kp.heat_a[fc] * p[k] + kp.heat_b[fc];
      const uint32_t e = in ? gslot(k, (uint32_t)(n + off)) : gslot(ko, (uint32_t)n);
      st_mg<S, C>(sto, e, v);
    }
  });
  if constexpr (GEN) scatter_faces<Lat, ODD, RAW, S, C>(kp, sto, n, nb, h, p, M, seed);
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = (w > v || w != w) ? w : v;
  }
  return v;
}

// Deterministic block reduction of NV values: a sum, or a max (NaN-propagating)
// for the entries whose bit is set in maxmask; result valid in thread 0.
// blockDim.x is a multiple of 64 and <= kMaxBlock.
__device__ __forceinline__ double pick_max(double a, double b) { return (b > a || b != b) ? b : a; }

template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], unsigned maxmask) {
  __shared__ double sh[kMaxBlock / 64][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = ((maxmask >> j) & 1u) ? wave_max(v[j]) : wave_sum(v[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) sh[wid][j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double a = sh[0][j];
      for (int w = 1; w < nw; ++w) a = ((maxmask >> j) & 1u) ? pick_max(a, sh[w][j]) : a + sh[w][j];
      v[j] = a;
    }
  }
}

// ------------------------------------------------------------------ step
enum : int { kModePlain = 0, kModeSnapshot = 1, kModeCompare = 2, kModeSpan = 3 };
constexpr int kPartStride = 8;  // doubles per block in the partials buffer

// One fused time step of the nodes of one block (block index lb of the lattice).
//   MODE 1 also stores u and T of the pre-collision state into snap (4 planes of n);
//   MODE 2 also accumulates, per block, sum|u - u_snap|^2, sum|u|^2,
//   sum (theta - theta_snap)^2, sum theta^2 and max|u| into part[lb];
//   MODE 3 does both: it compares with the snapshot, then replaces it.
// The per-node body of a step: gather, moments, residual bookkeeping,
// collisions, scatter.  G selects the general wall rules; seed (a hash of the
// lattice's step count) drives the stochastic rounding of FP16 storage.
template <class Lat, class S, class C, bool ODD, int MODE, bool G, bool SEP = false>
__device__ __forceinline__ void step_node(const KParams<C>& kp, const S& state, C* __restrict__ snap, int n,
                                          const Nbr& nb, double (&red)[5], uint32_t seed) {
  C h[Lat::Q], p[7];
  // A wavefront that is issuing its loads goes before wavefronts that are
  // computing, so the loads of the next wavefronts are in flight sooner.
  // Measured: FP16 storage 3-4 % faster; FP64 (2-3 wavefronts
  // per SIMD) 0.8-0.9 % faster; FP32 storage 0.7-0.9 % faster in the even
  // step but 1.5 % slower in the odd step, whose loads reach neighbour tiles.
  constexpr bool kLoadPriority =
      kStochastic<S> || std::is_same<C, double>::value || (!ODD && std::is_same<C, float>::value);
  if constexpr (kLoadPriority) __builtin_amdgcn_s_setprio(1);
  gather<Lat, ODD, G, S, C, SEP, true>(kp, state, n, nb, h, p);
  if constexpr (kLoadPriority) __builtin_amdgcn_s_setprio(0);
  const Pairs<Lat, C> P = make_pairs<Lat, C>(h);
  const Macro<C> M = macro<Lat, kFlowScale<S>, C>(kp, P, p);
  LBM_GLOBAL C* sn = gbl(snap);
  if constexpr (MODE == kModeCompare || MODE == kModeSpan) {
    const double ux = M.ux, uy = M.uy, uz = M.uz, T = M.T;
    const double dx = ux - (double)sn[n], dy = uy - (double)sn[n + kp.n], dz = uz - (double)sn[n + 2 * kp.n];
    const double dT = (T - (double)sn[n + 3 * kp.n]) * (double)kp.inv_dT;
    const double th = (T - (double)kp.T_ref) * (double)kp.inv_dT + 0.5;
    const double uu = ux * ux + uy * uy + uz * uz;
    red[0] = dx * dx + dy * dy + dz * dz;
    red[1] = uu;
    red[2] = dT * dT;
    red[3] = th * th;
    red[4] = sqrt(uu);
  }
  if constexpr (MODE == kModeSnapshot || MODE == kModeSpan) {
    sn[n] = M.ux;
    sn[n + kp.n] = M.uy;
    sn[n + 2 * kp.n] = M.uz;
    sn[n + 3 * kp.n] = M.T;
  }
  collide_flow<Lat, C>(kp, M, P, h);
  collide_heat<C>(kp, M, p);
  scatter<Lat, ODD, G, S, C, SEP, true>(kp, state, n, nb, h, p, M, seed);
}

// Node (x, y, z) lies on a face that moves or is open.
template <class C>
__device__ __forceinline__ bool on_special_face(const KParams<C>& kp, int x, int y, int z) {
  const int s = kp.special;
  return ((s & 1) && x == 0) || ((s & 2) && x == kp.nx - 1) || ((s & 4) && y == 0) ||
         ((s & 8) && y == kp.ny - 1) || ((s & 16) && z == 0) || ((s & 32) && z == kp.nz - 1);
}

// One fused time step of the nodes of one block (block index lb of the lattice).
//   MODE 1 also stores u and T of the pre-collision state into snap (4 planes of n);
//   MODE 2 also accumulates, per block, sum|u - u_snap|^2, sum|u|^2,
//   sum (theta - theta_snap)^2, sum theta^2 and max|u| into part[lb];
//   MODE 3 does both: it compares with the snapshot, then replaces it.
// With GEN the general wall rules run only in wavefronts that hold a node on a
// moving or open face; every other wavefront takes the lean rules, which give
// the same result for its nodes.  The choice is uniform per wavefront.  With
// SEP (separable tiles, odd step) both take their link indices from per-axis
// deltas: the same indices with fewer instructions.
template <class Lat, class S, class C, bool ODD, int MODE, bool GEN, bool SEP = false>
__device__ __forceinline__ void step_block(const KParams<C>& kp, const S& state, C* __restrict__ snap,
                                           double* __restrict__ part, int lb, uint32_t seed) {
  const int n = lb * blockDim.x + threadIdx.x;
  double red[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (n < kp.n) {
    int x, y, z;
    node_coords(kp, n, x, y, z);
    const Nbr nb = make_nbr(kp, x, y, z);
    if constexpr (GEN) {
      if (__ballot(on_special_face(kp, x, y, z)) != 0)
        step_node<Lat, S, C, ODD, MODE, true, SEP && ODD>(kp, state, snap, n, nb, red, seed);
      else
        step_node<Lat, S, C, ODD, MODE, false, SEP && ODD>(kp, state, snap, n, nb, red, seed);
    } else {
      step_node<Lat, S, C, ODD, MODE, false, SEP && ODD>(kp, state, snap, n, nb, red, seed);
    }
  }
  if constexpr (MODE == kModeCompare || MODE == kModeSpan) {
    block_reduce<5>(red, 1u << 4);
    if (threadIdx.x == 0) {
      LBM_GLOBAL double* pt = gbl(part);
#pragma unroll
      for (int j = 0; j < 5; ++j) pt[(size_t)lb * kPartStride + j] = red[j];
    }
  }
}

// First stage of the two-stage reduction of per-block partials: block b folds
// partials [b*blockDim, (b+1)*blockDim) into out[b] (sums; max for maxmask bits).
__global__ void __launch_bounds__(kMaxBlock) k_fold_partials(const double* __restrict__ in, int count,
                                                             unsigned maxmask, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < count) {
#pragma unroll
    for (int j = 0; j < 5; ++j) v[j] = in[(size_t)i * kPartStride + j];
  }
  block_reduce<5>(v, maxmask);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 5; ++j) out[(size_t)blockIdx.x * kPartStride + j] = v[j];
  }
}

// Forms the residual from the folded sums (sum|du|^2, sum|u|^2, sum dtheta^2,
// sum theta^2, max|u|): res[0] = r, res[1] = unstable (0/1), res[2..6] = the sums;
// res[7] (sticky) is set when unstable.
__device__ __forceinline__ void finish_residual(const double (&v)[5], double* __restrict__ res) {
  auto ratio = [](double num, double den) {
    if (den > 0.0) return sqrt(num / den);
    return num == 0.0 ? 0.0 : __builtin_inf();
  };
  const double ru = ratio(v[0], v[1]);
  const double rt = ratio(v[2], v[3]);
  double r = ru > rt ? ru : rt;
  bool bad = false;
#pragma unroll
  for (int j = 0; j < 5; ++j) bad = bad || !(v[j] == v[j]) || __builtin_isinf(v[j]);
  bad = bad || v[4] > 0.5;
  if (r != r) bad = true;
  res[0] = r;
  res[1] = bad ? 1.0 : 0.0;
#pragma unroll
  for (int j = 0; j < 5; ++j) res[2 + j] = v[j];
  if (bad) res[7] = 1.0;
}

// Second stage for a compare step: folds the first-stage partials and forms the
// residual.  res[0] = r, res[1] = unstable (0/1), res[2..6] = the five totals;
// res[7] (sticky) is set when unstable.
__global__ void __launch_bounds__(kMaxBlock) k_residual_final(const double* __restrict__ part, int count,
                                                              double* __restrict__ res) {
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < count; b += blockDim.x) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] += part[(size_t)b * kPartStride + j];
    v[4] = pick_max(v[4], part[(size_t)b * kPartStride + 4]);
  }
  block_reduce<5>(v, 1u << 4);
  if (threadIdx.x == 0) finish_residual(v, res);
}

// ------------------------------------------------------------------ init
__device__ __forceinline__ uint64_t splitmix64(uint64_t s) {
  // SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): one output from state s
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct InitArgs {
  int init_axis;
  double T_lo, T_hi;
  uint64_t seed;
  double noise_amp;
  double u[3];
};

// Initial state f = f^eq(rho0, u0) (Eq. 24 / 18) and g = g^eq(T, u0) (Eq. 42),
// T linear along init_axis plus counter-based uniform noise, stored shifted:
// h_i = w_i rho0 [e.u/cs^2 + (e.u)^2/(2 phi cs^4) - u^2/(2 phi cs^2)],
// p_k = omega_k [sigma (T - T_ref) + T e.u / csT^2].
template <class Lat, class S, class C>
__global__ void __launch_bounds__(kMaxBlock) k_init(const KParams<C> kp, const InitArgs ia, const S state) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  int c[3];
  node_coords(kp, n, c[0], c[1], c[2]);
  const int dim[3] = {kp.nx, kp.ny, kp.nz};
  double T = (double)kp.T_ref;
  if (ia.init_axis >= 0) {
    const double s = ((double)c[ia.init_axis] + 0.5) / (double)dim[ia.init_axis];
    T = ia.T_lo + (ia.T_hi - ia.T_lo) * s;
  }
  const double r = (double)(splitmix64(ia.seed ^ (uint64_t)n) >> 11) * (1.0 / 9007199254740992.0);
  const double noise = ia.noise_amp * (2.0 * r - 1.0);
  T = T + noise;
  const double phi = (double)kp.phi;
  const double uu = ia.u[0] * ia.u[0] + ia.u[1] * ia.u[1] + ia.u[2] * ia.u[2];
  static_for<0, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const double eu = Lat::e(0, i) * ia.u[0] + Lat::e(1, i) * ia.u[1] + Lat::e(2, i) * ia.u[2];
    const double v = weight<Lat, i>() * (3.0 * eu + 4.5 * eu * eu / phi - 1.5 * uu / phi);
    if constexpr (i == 0) st_f0<S, C>(state, (uint32_t)n, C(v));
    else st_mf<S, C>(state, fslot<Lat>(i, (uint32_t)n), C(v));
  });
  const double dsT = (double)kp.sigma * (T - (double)kp.T_ref);
  const double vp = (double)kp.varpi;
  const double csT2 = vp / 3.0;
  st_g0<S, C>(state, (uint32_t)n, C((1.0 - vp) * dsT));
  static_for<1, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const double eu = D3Q7::e(0, k) * ia.u[0] + D3Q7::e(1, k) * ia.u[1] + D3Q7::e(2, k) * ia.u[2];
    st_mg<S, C>(state, gslot(k, (uint32_t)n), C(vp / 6.0 * (dsT + T * eu / csT2)));
  });
}

// ------------------------------------------------------------------ fields
// Nodes [n0, n0 + count) of the lattice; output element n - n0 holds node n.
template <class Lat, class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_fields(const KParams<C> kp, const S state, int n0, int count,
                                                      double* rho, double* ux, double* uy, double* uz,
                                                      double* T) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  const int n = n0 + m;
  int x, y, z;
  node_coords(kp, n, x, y, z);
  const Nbr nb = make_nbr(kp, x, y, z);
  C h[Lat::Q], p[7];
  gather<Lat, ODD, true, S, C>(kp, state, n, nb, h, p);
  const Macro<C> M = macro<Lat, 1, C>(kp, make_pairs<Lat, C>(h), p);
  if (rho) rho[m] = 1.0 + (double)M.drho;
  if (ux) ux[m] = (double)M.ux;
  if (uy) uy[m] = (double)M.uy;
  if (uz) uz[m] = (double)M.uz;
  if (T) T[m] = (double)M.T;
}

// Per-block FP64 sums of (rho - rho0) and sigma (T - T_ref) of the current state.
template <class Lat, class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_totals(const KParams<C> kp, const S state,
                                                      double* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (n < kp.n) {
    int x, y, z;
    node_coords(kp, n, x, y, z);
    const Nbr nb = make_nbr(kp, x, y, z);
    C h[Lat::Q], p[7];
    gather<Lat, ODD, true, S, C>(kp, state, n, nb, h, p);
    for (int i = 0; i < Lat::Q; ++i) v[0] += (double)h[i];
    for (int k = 0; k < 7; ++k) v[1] += (double)p[k];
  }
  block_reduce<2>(v, 0u);
  if (threadIdx.x == 0) {
    part[(size_t)blockIdx.x * kPartStride + 0] = v[0];
    part[(size_t)blockIdx.x * kPartStride + 1] = v[1];
  }
}

// Second stage for the totals: folds the first-stage partials (two sums).
__global__ void __launch_bounds__(kMaxBlock) k_sum_final(const double* __restrict__ part, int count,
                                                         double* __restrict__ out) {
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < count; b += blockDim.x) {
    v[0] += part[(size_t)b * kPartStride + 0];
    v[1] += part[(size_t)b * kPartStride + 1];
  }
  block_reduce<2>(v, 0u);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[1];
  }
}

// Heat entering through each isothermal face during the last streaming, in
// two deterministic stages.  k_wall_flux: block (b, f) sums, in FP64, 2 g_k -
// 2 omega_k sigma T_w over chunk b (of gridDim.x equal chunks) of face f's
// wall nodes, k the population entering the fluid, into part[f * gridDim.x +
// b]; k_wall_fold adds each face's chunk sums in order into out[face].  The
// wall term 2 omega_k sigma T_w is taken as the step applies it, in the step's
// precision: the sum is then exactly the heat the discrete model exchanges
// with the wall.  (At Ra = 1e6 the flux per node is about 1/700 of a
// population, and the FP32 rounding of the wall term alone would move Nu by
// 4e-5.)
template <class Lat, class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_wall_flux(const KParams<C> kp, const S state,
                                                         const int* __restrict__ isothermal,
                                                         double* __restrict__ part) {
  const int face = blockIdx.y;
  const int a = face >> 1, side = face & 1;
  const int dim[3] = {kp.nx, kp.ny, kp.nz};
  const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
  const int cnt = dim[a1] * dim[a2];
  const int per = (cnt + (int)gridDim.x - 1) / (int)gridDim.x;
  const int m0 = (int)blockIdx.x * per, m1 = min(cnt, m0 + per);
  double v[1] = {0.0};
  if (isothermal[face]) {
    const int k = 1 + 2 * a + side;  // D3Q7 direction pointing into the fluid
    const double shift = (double)kp.heat_b[face];
    for (int m = m0 + (int)threadIdx.x; m < m1; m += blockDim.x) {
      int c[3];
      c[a] = side ? dim[a] - 1 : 0;
      c[a1] = m % dim[a1];
      c[a2] = m / dim[a1];
      const int n = c[0] + kp.nx * (c[1] + kp.ny * c[2]);
      double pk;
      if (!ODD) {
        pk = (double)ld_mg<S, C>(state, gslot(k, (uint32_t)n));
      } else {
        // the population enters from outside: anti-bounce-back of slot k of this node
        pk = (double)(kp.heat_a[face] * ld_mg<S, C>(state, gslot(k, (uint32_t)n)) + kp.heat_b[face]);
      }
      v[0] += 2.0 * pk - shift;
    }
  }
  block_reduce<1>(v, 0u);
  if (threadIdx.x == 0) part[face * (int)gridDim.x + (int)blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(64) k_wall_fold(const double* __restrict__ part, int chunks,
                                                  double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < chunks; ++b) s += part[blockIdx.x * chunks + b];
  out[blockIdx.x] = s;
}

// ------------------------------------------------------------------ state I/O
template <class Lat, class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_get_state(const KParams<C> kp, const S state,
                                                         double* f_out, double* g_out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  int x, y, z;
  node_coords(kp, n, x, y, z);
  const Nbr nb = make_nbr(kp, x, y, z);
  C h[Lat::Q], p[7];
  gather<Lat, ODD, true, S, C>(kp, state, n, nb, h, p);
  if (f_out) {
    static_for<0, Lat::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      f_out[(size_t)i * kp.n + n] = (double)h[i] + weight<Lat, i>();
    });
  }
  if (g_out) {
    const double vp = (double)kp.varpi, sT = (double)kp.sigma * (double)kp.T_ref;
    for (int k = 0; k < 7; ++k) {
      const double om = k == 0 ? 1.0 - vp : vp / 6.0;
      g_out[(size_t)k * kp.n + n] = (double)p[k] + om * sT;
    }
  }
}

// Sets slot `slot` of a lattice's step count (the slot the next step reads).
__global__ void __launch_bounds__(64) k_set_clock(uint32_t* clk, int slot, uint32_t value) {
  if (threadIdx.x == 0) gbl(clk)[slot] = value;
}

template <class Lat, class S, class C>
__global__ void __launch_bounds__(kMaxBlock) k_set_state(const KParams<C> kp, const S state,
                                                         const double* f_in, const double* g_in) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  static_for<0, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const C v = C(f_in[(size_t)i * kp.n + n] - weight<Lat, i>());
    if constexpr (i == 0) st_f0<S, C>(state, (uint32_t)n, v);
    else st_mf<S, C>(state, fslot<Lat>(i, (uint32_t)n), v);
  });
  const double vp = (double)kp.varpi, sT = (double)kp.sigma * (double)kp.T_ref;
  for (int k = 0; k < 7; ++k) {
    const double om = k == 0 ? 1.0 - vp : vp / 6.0;
    const C v = C(g_in[(size_t)k * kp.n + n] - om * sT);
    if (k == 0) st_g0<S, C>(state, (uint32_t)n, v);
    else st_mg<S, C>(state, gslot(k, (uint32_t)n), v);
  }
}

// Copies the pre-collision state of lattice `src` (at parity ODD) into lattice
// `dst` of the same shape and rest state, converting between storage types;
// dst is written in the even-parity layout.  Both store departures from the
// same rest state, so the copy is a plain conversion of each stored value.
template <class Lat, class SS, class CS, bool ODD, class SD, class CD>
__global__ void __launch_bounds__(kMaxBlock) k_transfer(const KParams<CS> kps, const SS src, const KParams<CD> kpd,
                                                        const SD dst) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kps.n) return;
  int x, y, z;
  node_coords(kps, n, x, y, z);
  const Nbr nb = make_nbr(kps, x, y, z);
  CS h[Lat::Q], p[7];
  gather<Lat, ODD, true, SS, CS>(kps, src, n, nb, h, p);
  static_for<0, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (i == 0) st_f0<SD, CD>(dst, (uint32_t)n, (CD)h[0]);
    else st_mf<SD, CD>(dst, fslot<Lat>(i, (uint32_t)n), (CD)h[i]);
  });
  st_g0<SD, CD>(dst, (uint32_t)n, (CD)p[0]);
#pragma unroll
  for (int k = 1; k < 7; ++k) st_mg<SD, CD>(dst, gslot(k, (uint32_t)n), (CD)p[k]);
}

}  // namespace lbm
