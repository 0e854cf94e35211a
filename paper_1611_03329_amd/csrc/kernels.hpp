// kernels.hpp -- gfx950 kernels of the fused DDF-MRT porous-convection step.
//
// Memory: ONE copy of the populations ("AA pattern"), population-major,
// plane k at state + k*pstride, node n = x + nx*(y + ny*z) inside a plane;
// f planes 0..Q-1 then g planes Q..Q+6.  Values are stored shifted by their
// rest state (see model.hpp).
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

#include "model.hpp"

namespace lbm {

constexpr int kMaxBlock = 256;

// ------------------------------------------------------------------ storage
template <class S, class C>
__device__ __forceinline__ C ld(const S* p) {
  return static_cast<C>(*p);
}
template <class S, class C>
__device__ __forceinline__ void st(S* p, C v) {
  *p = static_cast<S>(v);
}

// ------------------------------------------------------------------ geometry
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

// Link along velocity (ex, ey, ez) taken with sign `sg` (+1: to x + e, -1: to x - e).
struct Link {
  int off;
  bool in;
  int face;  // first wall face crossed (face order), valid when !in
};

template <int EX, int EY, int EZ, int SG>
__device__ __forceinline__ Link link(const Nbr& b) {
  Link L{0, true, 0};
  int face = -1;
  auto axis = [&](auto A, int e) {
    constexpr int a = decltype(A)::value;
    if (e == 0) return;
    const int side = (e * SG > 0) ? 1 : 0;
    L.off += b.off[a][side];
    if (!b.in[a][side]) {
      L.in = false;
      if (face < 0) face = 2 * a + side;
    }
  };
  axis(std::integral_constant<int, 0>{}, EX);
  axis(std::integral_constant<int, 1>{}, EY);
  axis(std::integral_constant<int, 2>{}, EZ);
  L.face = face < 0 ? 0 : face;
  return L;
}

// Moving-wall term of bounce-back for the population entering along direction j:
// 2 w_j rho0 (e_j . u_w) / cs^2 = 6 w_j (e_j . u_w).
template <class Lat, int J, class C>
__device__ __forceinline__ C wall_term(const KParams<C>& kp, int face) {
  constexpr int ex = Lat::e(0, J), ey = Lat::e(1, J), ez = Lat::e(2, J);
  C uw[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C v = kp.u_wall[0][a];
#pragma unroll
    for (int f = 1; f < 6; ++f) v = face == f ? kp.u_wall[f][a] : v;
    uw[a] = v;
  }
  C w6;
  if constexpr (Lat::Q == 19) w6 = C(6.0 * Lat::w36(J) / 36.0);
  else w6 = C(6.0 * Lat::w72(J) / 72.0);
  return w6 * (C(ex) * uw[0] + C(ey) * uw[1] + C(ez) * uw[2]);
}

// ------------------------------------------------------------------ gather
// Pre-collision shifted populations of node n at the current parity.
template <class Lat, bool ODD, class S, class C>
__device__ __forceinline__ void gather(const KParams<C>& kp, const S* __restrict__ st_, int n,
                                       const Nbr& nb, C (&h)[Lat::Q], C (&p)[7]) {
  const S* f = st_;
  const S* g = st_ + (size_t)Lat::Q * kp.pstride;
  static_for<0, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (!ODD) {
      h[i] = ld<S, C>(f + (size_t)i * kp.pstride + n);
    } else {
      constexpr int io = Lat::opp(i);
      const Link L = link<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), -1>(nb);
      const S* src = L.in ? (f + (size_t)io * kp.pstride + (n + L.off)) : (f + (size_t)i * kp.pstride + n);
      C v = ld<S, C>(src);
      if constexpr (i != 0) {
        if (kp.moving && !L.in) v += wall_term<Lat, i>(kp, L.face);
      }
      h[i] = v;
    }
  });
  static_for<0, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if constexpr (!ODD) {
      p[k] = ld<S, C>(g + (size_t)k * kp.pstride + n);
    } else {
      constexpr int ko = D3Q7::opp(k);
      const Link L = link<D3Q7::e(0, k), D3Q7::e(1, k), D3Q7::e(2, k), -1>(nb);
      const S* src = L.in ? (g + (size_t)ko * kp.pstride + (n + L.off)) : (g + (size_t)k * kp.pstride + n);
      C v = ld<S, C>(src);
      if constexpr (k != 0) {
        if (!L.in) v = kp.heat_a[L.face] * v + kp.heat_b[L.face];
      }
      p[k] = v;
    }
  });
}

// ------------------------------------------------------------------ scatter
// Post-collision shifted populations of node n, written for the next parity.
template <class Lat, bool ODD, class S, class C>
__device__ __forceinline__ void scatter(const KParams<C>& kp, S* __restrict__ st_, int n, const Nbr& nb,
                                        const C (&h)[Lat::Q], const C (&p)[7]) {
  S* f = st_;
  S* g = st_ + (size_t)Lat::Q * kp.pstride;
  static_for<0, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int io = Lat::opp(i);
    if constexpr (!ODD) {
      st<S, C>(f + (size_t)io * kp.pstride + n, h[i]);
    } else {
      const Link L = link<Lat::e(0, i), Lat::e(1, i), Lat::e(2, i), +1>(nb);
      C v = h[i];
      if constexpr (i != 0) {
        if (kp.moving && !L.in) v += wall_term<Lat, io>(kp, L.face);
      }
      S* dst = L.in ? (f + (size_t)i * kp.pstride + (n + L.off)) : (f + (size_t)io * kp.pstride + n);
      st<S, C>(dst, v);
    }
  });
  static_for<0, 7>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int ko = D3Q7::opp(k);
    if constexpr (!ODD) {
      st<S, C>(g + (size_t)ko * kp.pstride + n, p[k]);
    } else {
      const Link L = link<D3Q7::e(0, k), D3Q7::e(1, k), D3Q7::e(2, k), +1>(nb);
      C v = p[k];
      if constexpr (k != 0) {
        if (!L.in) v = kp.heat_a[L.face] * v + kp.heat_b[L.face];
      }
      S* dst = L.in ? (g + (size_t)k * kp.pstride + (n + L.off)) : (g + (size_t)ko * kp.pstride + n);
      st<S, C>(dst, v);
    }
  });
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
enum : int { kModePlain = 0, kModeSnapshot = 1, kModeCompare = 2 };
constexpr int kPartStride = 8;  // doubles per block in the partials buffer

// One fused time step for every node.
//   MODE 1 also stores u and T of the pre-collision state into snap (4 planes of n);
//   MODE 2 also accumulates, per block, sum|u - u_snap|^2, sum|u|^2,
//   sum (theta - theta_snap)^2, sum theta^2 and max|u| into part.
template <class Lat, class S, class C, bool ODD, int MODE>
__global__ void __launch_bounds__(kMaxBlock) k_step(const KParams<C> kp, S* __restrict__ state,
                                                    C* __restrict__ snap, double* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double red[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (n < kp.n) {
    const int x = n % kp.nx;
    const int yz = n / kp.nx;
    const int y = yz % kp.ny;
    const int z = yz / kp.ny;
    const Nbr nb = make_nbr(kp, x, y, z);
    C h[Lat::Q], p[7];
    gather<Lat, ODD, S, C>(kp, state, n, nb, h, p);
    const Macro<C> M = macro<Lat, C>(kp, h, p);
    if constexpr (MODE == kModeSnapshot) {
      snap[n] = M.ux;
      snap[n + kp.n] = M.uy;
      snap[n + 2 * kp.n] = M.uz;
      snap[n + 3 * kp.n] = M.T;
    }
    if constexpr (MODE == kModeCompare) {
      const double ux = M.ux, uy = M.uy, uz = M.uz, T = M.T;
      const double dx = ux - (double)snap[n], dy = uy - (double)snap[n + kp.n],
                   dz = uz - (double)snap[n + 2 * kp.n];
      const double dT = (T - (double)snap[n + 3 * kp.n]) * (double)kp.inv_dT;
      const double th = (T - (double)kp.T_ref) * (double)kp.inv_dT + 0.5;
      const double uu = ux * ux + uy * uy + uz * uz;
      red[0] = dx * dx + dy * dy + dz * dz;
      red[1] = uu;
      red[2] = dT * dT;
      red[3] = th * th;
      red[4] = sqrt(uu);
    }
    collide_flow<Lat, C>(kp, M, h);
    collide_heat<C>(kp, M, p);
    scatter<Lat, ODD, S, C>(kp, state, n, nb, h, p);
  }
  if constexpr (MODE == kModeCompare) {
    block_reduce<5>(red, 1u << 4);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < 5; ++j) part[(size_t)blockIdx.x * kPartStride + j] = red[j];
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
  if (threadIdx.x == 0) {
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
};

// Rest state f = f^eq(rho0, 0) (h = 0) and g = g^eq(T, 0) = omega_k sigma T
// (Eq. 42), T linear along init_axis plus counter-based uniform noise.
template <class Lat, class S, class C>
__global__ void __launch_bounds__(kMaxBlock) k_init(const KParams<C> kp, const InitArgs ia, S* __restrict__ state) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  const int c[3] = {n % kp.nx, (n / kp.nx) % kp.ny, n / kp.nxy};
  const int dim[3] = {kp.nx, kp.ny, kp.nz};
  double T = (double)kp.T_ref;
  if (ia.init_axis >= 0) {
    const double s = ((double)c[ia.init_axis] + 0.5) / (double)dim[ia.init_axis];
    T = ia.T_lo + (ia.T_hi - ia.T_lo) * s;
  }
  const double r = (double)(splitmix64(ia.seed ^ (uint64_t)n) >> 11) * (1.0 / 9007199254740992.0);
  const double noise = ia.noise_amp * (2.0 * r - 1.0);
  T = T + noise;
  S* f = state;
  S* g = state + (size_t)Lat::Q * kp.pstride;
  for (int i = 0; i < Lat::Q; ++i) st<S, C>(f + (size_t)i * kp.pstride + n, C(0));
  const double dsT = (double)kp.sigma * (T - (double)kp.T_ref);
  const double vp = (double)kp.varpi;
  st<S, C>(g + n, C((1.0 - vp) * dsT));
  for (int k = 1; k < 7; ++k) st<S, C>(g + (size_t)k * kp.pstride + n, C(vp / 6.0 * dsT));
}

// ------------------------------------------------------------------ fields
template <class Lat, class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_fields(const KParams<C> kp, const S* __restrict__ state,
                                                      double* rho, double* ux, double* uy, double* uz,
                                                      double* T) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  const int x = n % kp.nx, yz = n / kp.nx, y = yz % kp.ny, z = yz / kp.ny;
  const Nbr nb = make_nbr(kp, x, y, z);
  C h[Lat::Q], p[7];
  gather<Lat, ODD, S, C>(kp, state, n, nb, h, p);
  const Macro<C> M = macro<Lat, C>(kp, h, p);
  if (rho) rho[n] = 1.0 + (double)M.drho;
  if (ux) ux[n] = (double)M.ux;
  if (uy) uy[n] = (double)M.uy;
  if (uz) uz[n] = (double)M.uz;
  if (T) T[n] = (double)M.T;
}

// Per-block FP64 sums of (rho - rho0) and sigma (T - T_ref) of the current state.
template <class Lat, class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_totals(const KParams<C> kp, const S* __restrict__ state,
                                                      double* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (n < kp.n) {
    const int x = n % kp.nx, yz = n / kp.nx, y = yz % kp.ny, z = yz / kp.ny;
    const Nbr nb = make_nbr(kp, x, y, z);
    C h[Lat::Q], p[7];
    gather<Lat, ODD, S, C>(kp, state, n, nb, h, p);
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

// Heat entering through each isothermal face during the last streaming:
// one block per face, FP64 sum of 2 g_k - 2 omega_k sigma T_w over the face's
// wall nodes, k the population entering the fluid.  out[face] = that sum.
template <class Lat, class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_wall_flux(const KParams<C> kp, const S* __restrict__ state,
                                                         const int* __restrict__ isothermal,
                                                         const double* __restrict__ T_wall,
                                                         double* __restrict__ out) {
  const int face = blockIdx.x;
  const int a = face >> 1, side = face & 1;
  const int dim[3] = {kp.nx, kp.ny, kp.nz};
  const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
  const int cnt = dim[a1] * dim[a2];
  double v[1] = {0.0};
  if (isothermal[face]) {
    const int k = 1 + 2 * a + side;  // D3Q7 direction pointing into the fluid
    const double w = (double)kp.varpi / 6.0;
    const double shift = 2.0 * w * (double)kp.sigma * (T_wall[face] - (double)kp.T_ref);
    const S* g = state + (size_t)Lat::Q * kp.pstride;
    for (int m = threadIdx.x; m < cnt; m += blockDim.x) {
      int c[3];
      c[a] = side ? dim[a] - 1 : 0;
      c[a1] = m % dim[a1];
      c[a2] = m / dim[a1];
      const int n = c[0] + kp.nx * (c[1] + kp.ny * c[2]);
      double pk;
      if (!ODD) {
        pk = (double)ld<S, C>(g + (size_t)k * kp.pstride + n);
      } else {
        // the population enters from outside: anti-bounce-back of slot k of this node
        pk = (double)(kp.heat_a[face] * ld<S, C>(g + (size_t)k * kp.pstride + n) + kp.heat_b[face]);
      }
      v[0] += 2.0 * pk - shift;
    }
  }
  block_reduce<1>(v, 0u);
  if (threadIdx.x == 0) out[face] = v[0];
}

// ------------------------------------------------------------------ state I/O
template <class Lat, class S, class C, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_get_state(const KParams<C> kp, const S* __restrict__ state,
                                                         double* f_out, double* g_out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  const int x = n % kp.nx, yz = n / kp.nx, y = yz % kp.ny, z = yz / kp.ny;
  const Nbr nb = make_nbr(kp, x, y, z);
  C h[Lat::Q], p[7];
  gather<Lat, ODD, S, C>(kp, state, n, nb, h, p);
  if (f_out) {
    static_for<0, Lat::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      double w;
      if constexpr (Lat::Q == 19) w = Lat::w36(i) / 36.0;
      else w = Lat::w72(i) / 72.0;
      f_out[(size_t)i * kp.n + n] = (double)h[i] + w;
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

template <class Lat, class S, class C>
__global__ void __launch_bounds__(kMaxBlock) k_set_state(const KParams<C> kp, S* __restrict__ state,
                                                         const double* f_in, const double* g_in) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kp.n) return;
  S* f = state;
  S* g = state + (size_t)Lat::Q * kp.pstride;
  static_for<0, Lat::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    double w;
    if constexpr (Lat::Q == 19) w = Lat::w36(i) / 36.0;
    else w = Lat::w72(i) / 72.0;
    st<S, C>(f + (size_t)i * kp.pstride + n, C(f_in[(size_t)i * kp.n + n] - w));
  });
  const double vp = (double)kp.varpi, sT = (double)kp.sigma * (double)kp.T_ref;
  for (int k = 0; k < 7; ++k) {
    const double om = k == 0 ? 1.0 - vp : vp / 6.0;
    st<S, C>(g + (size_t)k * kp.pstride + n, C(g_in[(size_t)k * kp.n + n] - om * sT));
  }
}

}  // namespace lbm
