// lattice.hpp -- discrete velocity sets and moment bases of the DDF-MRT model
// (Liu & He, arXiv:1611.03329), as compile-time tables for the gfx950 kernels.
//
// The transformation matrices are not typed in as numbers here: each row is
// generated from the moment polynomial that the row stands for (the basis of
// Eq. 20 for D3Q19 and Eq. 13 for D3Q15, as defined in the paper's Ref. [49]),
// evaluated on the velocity set of Eq. 19 / Eq. 12.  The result equals the
// printed Eqs. A2 / A1.  The rows are mutually orthogonal, so the inverse is
// M^T diag(1/|M_k|^2).  The D3Q7 matrix N (Eq. 36) is not orthogonal and its
// inverse is the printed Eq. 43.
#pragma once

#include <type_traits>
#include <utility>

namespace lbm {

// Compile-time loop: calls f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, class F>
__host__ __device__ __forceinline__ constexpr void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(static_cast<F&&>(f));
  }
}

// Moment rows are even or odd under e -> -e; a direction i >= 1 whose opposite
// has a larger index represents its pair.
template <class Lat>
constexpr bool row_is_even(int k) {
  for (int i = 0; i < Lat::Q; ++i)
    if (Lat::moment(k, Lat::opp(i)) != Lat::moment(k, i)) return false;
  return true;
}
template <class Lat>
constexpr bool row_is_odd(int k) {
  for (int i = 0; i < Lat::Q; ++i)
    if (Lat::moment(k, Lat::opp(i)) != -Lat::moment(k, i)) return false;
  return true;
}
template <class Lat>
constexpr bool is_pair_rep(int i) { return i >= 1 && Lat::opp(i) > i; }

// ---------------------------------------------------------------- D3Q19
struct D3Q19 {
  static constexpr int Q = 19;
  // Eq. 19
  static constexpr int E[3][19] = {
      {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
      {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
      {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1}};

  static constexpr int e(int a, int i) { return E[a][i]; }
  static constexpr int r2(int i) { return e(0, i) * e(0, i) + e(1, i) * e(1, i) + e(2, i) * e(2, i); }

  // weights of Eq. 24, as exact fractions num/36
  static constexpr int w36(int i) { return r2(i) == 0 ? 12 : (r2(i) == 1 ? 2 : 1); }

  // Moment k of the basis (rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww,
  // piww, pxy, pyz, pzx, mx, my, mz) evaluated on velocity i.
  static constexpr int moment(int k, int i) {
    const int x = e(0, i), y = e(1, i), z = e(2, i), s = r2(i);
    switch (k) {
      case 0: return 1;
      case 1: return 19 * s - 30;
      case 2: return (21 * s * s - 53 * s + 24) / 2;
      case 3: return x;
      case 4: return (5 * s - 9) * x;
      case 5: return y;
      case 6: return (5 * s - 9) * y;
      case 7: return z;
      case 8: return (5 * s - 9) * z;
      case 9: return 3 * x * x - s;
      case 10: return (3 * s - 5) * (3 * x * x - s);
      case 11: return y * y - z * z;
      case 12: return (3 * s - 5) * (y * y - z * z);
      case 13: return x * y;
      case 14: return y * z;
      case 15: return z * x;
      case 16: return (y * y - z * z) * x;
      case 17: return (z * z - x * x) * y;
      default: return (x * x - y * y) * z;
    }
  }
  static constexpr int norm2(int k) {
    int n = 0;
    for (int i = 0; i < Q; ++i) n += moment(k, i) * moment(k, i);
    return n;
  }
  static constexpr int opp(int i) {
    for (int j = 0; j < Q; ++j)
      if (e(0, j) == -e(0, i) && e(1, j) == -e(1, i) && e(2, j) == -e(2, i)) return j;
    return -1;
  }
};

// ---------------------------------------------------------------- D3Q15
struct D3Q15 {
  static constexpr int Q = 15;
  // Eq. 12
  static constexpr int E[3][15] = {
      {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
      {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
      {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1}};

  static constexpr int e(int a, int i) { return E[a][i]; }
  static constexpr int r2(int i) { return e(0, i) * e(0, i) + e(1, i) * e(1, i) + e(2, i) * e(2, i); }

  // weights of Eq. 18 as num/72
  static constexpr int w72(int i) { return r2(i) == 0 ? 16 : (r2(i) == 1 ? 8 : 1); }

  // Moment k of (rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, pww, pxy, pyz, pzx, mxyz).
  static constexpr int moment(int k, int i) {
    const int x = e(0, i), y = e(1, i), z = e(2, i), s = r2(i);
    switch (k) {
      case 0: return 1;
      case 1: return s - 2;
      case 2: return (15 * s * s - 55 * s + 32) / 2;
      case 3: return x;
      case 4: return (5 * s - 13) / 2 * x;
      case 5: return y;
      case 6: return (5 * s - 13) / 2 * y;
      case 7: return z;
      case 8: return (5 * s - 13) / 2 * z;
      case 9: return 3 * x * x - s;
      case 10: return y * y - z * z;
      case 11: return x * y;
      case 12: return y * z;
      case 13: return z * x;
      default: return x * y * z;
    }
  }
  static constexpr int norm2(int k) {
    int n = 0;
    for (int i = 0; i < Q; ++i) n += moment(k, i) * moment(k, i);
    return n;
  }
  static constexpr int opp(int i) {
    for (int j = 0; j < Q; ++j)
      if (e(0, j) == -e(0, i) && e(1, j) == -e(1, i) && e(2, j) == -e(2, i)) return j;
    return -1;
  }
};

// ---------------------------------------------------------------- D3Q7
struct D3Q7 {
  static constexpr int Q = 7;
  static constexpr int E[3][7] = {{0, 1, -1, 0, 0, 0, 0}, {0, 0, 0, 1, -1, 0, 0}, {0, 0, 0, 0, 0, 1, -1}};
  static constexpr int e(int a, int i) { return E[a][i]; }
  // Eq. 36: rows 1, e_x, e_y, e_z, |e|^2, e_x^2 - e_y^2, e_x^2 - e_z^2
  static constexpr int N(int k, int i) {
    const int x = e(0, i), y = e(1, i), z = e(2, i);
    switch (k) {
      case 0: return 1;
      case 1: return x;
      case 2: return y;
      case 3: return z;
      case 4: return x * x + y * y + z * z;
      case 5: return x * x - y * y;
      default: return x * x - z * z;
    }
  }
  // Eq. 43, times 6 so that every entry is an integer
  static constexpr int Ninv6[7][7] = {{6, 0, 0, 0, -6, 0, 0},  {0, 3, 0, 0, 1, 1, 1},
                                      {0, -3, 0, 0, 1, 1, 1},  {0, 0, 3, 0, 1, -2, 1},
                                      {0, 0, -3, 0, 1, -2, 1}, {0, 0, 0, 3, 1, 1, -2},
                                      {0, 0, 0, -3, 1, 1, -2}};
  static constexpr int opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }
};

// Compile-time checks of the generated tables against facts of the paper.
namespace detail {
constexpr bool check_d3q19() {
  // Eq. A2 row norms and two printed rows
  constexpr int norms[19] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8};
  for (int k = 0; k < 19; ++k)
    if (D3Q19::norm2(k) != norms[k]) return false;
  constexpr int row2[19] = {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
  constexpr int row17[19] = {0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  for (int i = 0; i < 19; ++i)
    if (D3Q19::moment(2, i) != row2[i] || D3Q19::moment(17, i) != row17[i]) return false;
  // orthogonality
  for (int a = 0; a < 19; ++a)
    for (int b = a + 1; b < 19; ++b) {
      int s = 0;
      for (int i = 0; i < 19; ++i) s += D3Q19::moment(a, i) * D3Q19::moment(b, i);
      if (s != 0) return false;
    }
  int wsum = 0;
  for (int i = 0; i < 19; ++i) wsum += D3Q19::w36(i);
  return wsum == 36;
}
constexpr bool check_d3q15() {
  constexpr int norms[15] = {15, 18, 360, 10, 40, 10, 40, 10, 40, 12, 4, 8, 8, 8, 8};
  for (int k = 0; k < 15; ++k)
    if (D3Q15::norm2(k) != norms[k]) return false;
  for (int a = 0; a < 15; ++a)
    for (int b = a + 1; b < 15; ++b) {
      int s = 0;
      for (int i = 0; i < 15; ++i) s += D3Q15::moment(a, i) * D3Q15::moment(b, i);
      if (s != 0) return false;
    }
  int wsum = 0;
  for (int i = 0; i < 15; ++i) wsum += D3Q15::w72(i);
  return wsum == 72;
}
constexpr bool check_d3q7() {
  for (int a = 0; a < 7; ++a)
    for (int b = 0; b < 7; ++b) {
      int s = 0;
      for (int i = 0; i < 7; ++i) s += D3Q7::N(a, i) * D3Q7::Ninv6[i][b];
      if (s != (a == b ? 6 : 0)) return false;
    }
  return true;
}
template <class Lat>
constexpr bool every_row_has_parity() {
  for (int k = 0; k < Lat::Q; ++k)
    if (!row_is_even<Lat>(k) && !row_is_odd<Lat>(k)) return false;
  return true;
}
static_assert(check_d3q19(), "D3Q19 moment basis does not reproduce Eq. A2");
static_assert(every_row_has_parity<D3Q19>() && every_row_has_parity<D3Q15>(),
              "a moment row is neither even nor odd");
static_assert(check_d3q15(), "D3Q15 moment basis does not reproduce Eq. A1");
static_assert(check_d3q7(), "N times the printed inverse is not the identity");
}  // namespace detail

}  // namespace lbm
