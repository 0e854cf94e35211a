/*
 * lbm_oracle.c -- plain, slow, FP64 CPU oracle of the REV-scale DDF-MRT lattice
 * Boltzmann model (Liu & He, arXiv:1611.03329).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.
 *
 * Every step follows the paper in its own order and notation:
 *   m = M f (Eq. 11), m* = m - Lambda (m - m^eq) + (I - Lambda/2) S~ (Eq. 9),
 *   f* = M^-1 m* (Eq. 10), streaming (Eq. 10);
 *   n = N g, n* = n - Q (n - n^eq) (Eq. 34), g* = N^-1 n* (Eq. 43), streaming (Eq. 35).
 * Matrices are the printed ones (Eqs. A1, A2, 36, 43) applied densely; M^-1 is
 * obtained by Gauss-Jordan elimination of the printed M.
 *
 * Readings of places where the paper is silent or garbled (each one is also
 * listed in the design notes):
 *   R1  Eq. 28 sums e_i f_i over i = 0..8 (a two-dimensional leftover); the sum
 *       runs over all q directions, as in Eq. 26.
 *   R2  Eq. 14 has rho F, Eq. 26 has rho0 F; the incompressible rho0 is used.
 *   R3  The equilibria of the conserved moments (rows 0, 3, 5, 7) are not listed;
 *       they are those of M f^eq: rho and rho0*u.
 *   R4  Eq. 51 prints s_nu where its inverse is meant (compare Eq. 56).
 *   R5  Walls: halfway bounce-back for f (plus the moving-wall term
 *       2 w_i rho0 e_i.u_w / cs^2), anti-bounce-back for isothermal g
 *       (g_k = -g*_kbar + 2 omega_k sigma T_w), bounce-back for adiabatic g.
 *       The paper itself used non-equilibrium extrapolation (Sec. 4).
 *       A link leaving through several wall faces takes the first of them in
 *       face order (-x,+x,-y,+y,-z,+z) for its wall velocity; a wall face
 *       takes precedence over an outlet face.  Outlets are open boundaries
 *       at rho0: the incoming population is the anti-bounce-back of the
 *       outgoing one to twice the even part of f^eq(rho0, u) (Eq. 24 / 18),
 *       f_ibar = -f*_i + 2 w_i rho0 [1 + (e.u)^2/(2 phi cs^4) - u^2/(2 phi cs^2)],
 *       with u the node's own velocity at the time of the collision; for g the
 *       same with the node's own temperature, g_kbar = -g*_k + 2 omega_k sigma T.
 *   R6  Buoyancy G = gbeta (T - T0) along +gravity_axis (hot fluid rises).
 *   R7  Halfway walls: L = n along length_axis, K = Da L^2.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- lattices */

/* Eq. 19: D3Q19 discrete velocities (columns) */
static const int E19[3][19] = {
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1}};

/* Eq. 12: D3Q15 discrete velocities; the first 7 columns are the D3Q7 set */
static const int E15[3][15] = {
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1}};

/* Eq. A2: D3Q19 transformation matrix */
static const double M19[19][19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},
    {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, -4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1}};

/* Eq. A1: D3Q15 transformation matrix */
static const double M15[15][15] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-2, -1, -1, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1},
    {16, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1},
    {0, 0, 0, 0, 0, -4, 4, 1, 1, 1, 1, -1, -1, -1, -1},
    {0, 2, 2, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1}};

/* Eq. 36: D3Q7 transformation matrix */
static const double N7[7][7] = {
    {1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0},
    {0, 0, 0, 0, 0, 1, -1},
    {0, 1, 1, 1, 1, 1, 1},
    {0, 1, 1, -1, -1, 0, 0},
    {0, 1, 1, 0, 0, -1, -1}};

/* Eq. 43: inverse of N as printed */
static const double N7INV[7][7] = {
    {1, 0, 0, 0, -1, 0, 0},
    {0, 0.5, 0, 0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0},
    {0, -0.5, 0, 0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0},
    {0, 0, 0.5, 0, 1.0 / 6.0, -1.0 / 3.0, 1.0 / 6.0},
    {0, 0, -0.5, 0, 1.0 / 6.0, -1.0 / 3.0, 1.0 / 6.0},
    {0, 0, 0, 0.5, 1.0 / 6.0, 1.0 / 6.0, -1.0 / 3.0},
    {0, 0, 0, -0.5, 1.0 / 6.0, 1.0 / 6.0, -1.0 / 3.0}};

static const double CS2 = 1.0 / 3.0; /* lattice sound speed squared, c = 1 */
static const double RHO0 = 1.0;      /* Sec. 4 default */

static int valid_q(int q) { return q == 19 || q == 15 || q == 7; }

static int evel(int q, int a, int i) {
  if (q == 19) return E19[a][i];
  return E15[a][i]; /* q = 15 or 7 (first seven columns of Eq. 12) */
}

int ref_velocities(int q, int* e) {
  if (!valid_q(q) || !e) return REF_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < q; ++i) e[a * q + i] = evel(q, a, i);
  return REF_OK;
}

/* weights: Eq. 24 (D3Q19), Eq. 18 (D3Q15), Eq. 42 (D3Q7, omega) */
int ref_weights(int q, double varpi, double* w) {
  if (!valid_q(q) || !w) return REF_ERR_INVALID_ARG;
  for (int i = 0; i < q; ++i) {
    int e2 = evel(q, 0, i) * evel(q, 0, i) + evel(q, 1, i) * evel(q, 1, i) +
             evel(q, 2, i) * evel(q, 2, i);
    if (q == 19)
      w[i] = (e2 == 0) ? 1.0 / 3.0 : (e2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
    else if (q == 15)
      w[i] = (e2 == 0) ? 2.0 / 9.0 : (e2 == 1) ? 1.0 / 9.0 : 1.0 / 72.0;
    else
      w[i] = (e2 == 0) ? 1.0 - varpi : varpi / 6.0;
  }
  return REF_OK;
}

static const double* matrix_ptr(int q) {
  if (q == 19) return &M19[0][0];
  if (q == 15) return &M15[0][0];
  return &N7[0][0];
}

int ref_matrix(int q, double* M) {
  if (!valid_q(q) || !M) return REF_ERR_INVALID_ARG;
  memcpy(M, matrix_ptr(q), sizeof(double) * q * q);
  return REF_OK;
}

/* X = A^-1 by Gauss-Jordan elimination with partial pivoting (n <= 19) */
static int gauss_jordan(int n, const double* A, double* X) {
  double a[19][38];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c)
      a[r][c] = (c < n) ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (a[piv][col] == 0.0) return REF_ERR_INVALID_ARG;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        double t = a[col][c];
        a[col][c] = a[piv][c];
        a[piv][c] = t;
      }
    double d = a[col][col];
    for (int c = 0; c < 2 * n; ++c) a[col][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double fct = a[r][col];
      if (fct == 0.0) continue;
      for (int c = 0; c < 2 * n; ++c) a[r][c] -= fct * a[col][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) X[r * n + c] = a[r][n + c];
  return REF_OK;
}

int ref_matrix_inverse(int q, double* Minv) {
  if (!valid_q(q) || !Minv) return REF_ERR_INVALID_ARG;
  if (q == 7) {
    memcpy(Minv, &N7INV[0][0], sizeof(double) * 49);
    return REF_OK;
  }
  return gauss_jordan(q, matrix_ptr(q), Minv);
}

/* Eq. 24 (D3Q19) and Eq. 18 (D3Q15) */
int ref_feq(int q, double rho, const double* u, double phi, double* feq) {
  if ((q != 19 && q != 15) || !u || !feq) return REF_ERR_INVALID_ARG;
  double w[19];
  ref_weights(q, 0.5, w);
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < q; ++i) {
    double eu = evel(q, 0, i) * u[0] + evel(q, 1, i) * u[1] + evel(q, 2, i) * u[2];
    feq[i] = w[i] * (rho + RHO0 * (eu / CS2 + eu * eu / (2.0 * phi * CS2 * CS2) -
                                   uu / (2.0 * phi * CS2)));
  }
  return REF_OK;
}

/* Eq. 21 (D3Q19, beta1 = 3, beta2 = -5.5, beta3 = -0.5) and Eq. 15 (D3Q15,
 * beta1 = 1, beta2 = -5); conserved rows 0, 3, 5, 7 per reading R3. */
int ref_meq(int q, double rho, const double* u, double phi, double* meq) {
  if ((q != 19 && q != 15) || !u || !meq) return REF_ERR_INVALID_ARG;
  const double ux = u[0], uy = u[1], uz = u[2];
  const double uu = ux * ux + uy * uy + uz * uz;
  if (q == 19) {
    const double b1 = 3.0, b2 = -5.5, b3 = -0.5;
    const double pxx3 = RHO0 * (2.0 * ux * ux - uy * uy - uz * uz) / phi; /* 3 p_xx^eq */
    const double pww = RHO0 * (uy * uy - uz * uz) / phi;
    meq[0] = rho;
    meq[1] = -11.0 * rho + 19.0 * RHO0 * uu / phi;
    meq[2] = b1 * rho + b2 * RHO0 * uu / phi;
    meq[3] = RHO0 * ux;
    meq[4] = -2.0 / 3.0 * RHO0 * ux;
    meq[5] = RHO0 * uy;
    meq[6] = -2.0 / 3.0 * RHO0 * uy;
    meq[7] = RHO0 * uz;
    meq[8] = -2.0 / 3.0 * RHO0 * uz;
    meq[9] = pxx3;
    meq[10] = b3 * pxx3; /* 3 pi_xx^eq = 3 beta3 p_xx^eq */
    meq[11] = pww;
    meq[12] = b3 * pww;
    meq[13] = RHO0 * ux * uy / phi;
    meq[14] = RHO0 * uy * uz / phi;
    meq[15] = RHO0 * uz * ux / phi;
    meq[16] = 0.0;
    meq[17] = 0.0;
    meq[18] = 0.0;
  } else {
    const double b1 = 1.0, b2 = -5.0;
    meq[0] = rho;
    meq[1] = -rho + RHO0 * uu / phi;
    meq[2] = b1 * rho + b2 * RHO0 * uu / phi;
    meq[3] = RHO0 * ux;
    meq[4] = -7.0 / 3.0 * RHO0 * ux;
    meq[5] = RHO0 * uy;
    meq[6] = -7.0 / 3.0 * RHO0 * uy;
    meq[7] = RHO0 * uz;
    meq[8] = -7.0 / 3.0 * RHO0 * uz;
    meq[9] = RHO0 * (2.0 * ux * ux - uy * uy - uz * uz) / phi;
    meq[10] = RHO0 * (uy * uy - uz * uz) / phi;
    meq[11] = RHO0 * ux * uy / phi;
    meq[12] = RHO0 * uy * uz / phi;
    meq[13] = RHO0 * uz * ux / phi;
    meq[14] = 0.0;
  }
  return REF_OK;
}

/* Eq. 23 (D3Q19) and Eq. 17 (D3Q15) */
int ref_forcing_moments(int q, const double* u, const double* F, double phi, double* S) {
  if ((q != 19 && q != 15) || !u || !F || !S) return REF_ERR_INVALID_ARG;
  const double ux = u[0], uy = u[1], uz = u[2];
  const double Fx = F[0], Fy = F[1], Fz = F[2];
  const double uF = ux * Fx + uy * Fy + uz * Fz;
  if (q == 19) {
    S[0] = 0.0;
    S[1] = 38.0 * RHO0 * uF / phi;
    S[2] = -11.0 * RHO0 * uF / phi;
    S[3] = RHO0 * Fx;
    S[4] = -2.0 / 3.0 * RHO0 * Fx;
    S[5] = RHO0 * Fy;
    S[6] = -2.0 / 3.0 * RHO0 * Fy;
    S[7] = RHO0 * Fz;
    S[8] = -2.0 / 3.0 * RHO0 * Fz;
    S[9] = 2.0 * RHO0 * (2.0 * ux * Fx - uy * Fy - uz * Fz) / phi;
    S[10] = -RHO0 * (2.0 * ux * Fx - uy * Fy - uz * Fz) / phi;
    S[11] = 2.0 * RHO0 * (uy * Fy - uz * Fz) / phi;
    S[12] = -RHO0 * (uy * Fy - uz * Fz) / phi;
    S[13] = RHO0 * (ux * Fy + uy * Fx) / phi;
    S[14] = RHO0 * (uy * Fz + uz * Fy) / phi;
    S[15] = RHO0 * (ux * Fz + uz * Fx) / phi;
    S[16] = 0.0;
    S[17] = 0.0;
    S[18] = 0.0;
  } else {
    S[0] = 0.0;
    S[1] = 2.0 * RHO0 * uF / phi;
    S[2] = -10.0 * RHO0 * uF / phi;
    S[3] = RHO0 * Fx;
    S[4] = -7.0 / 3.0 * RHO0 * Fx;
    S[5] = RHO0 * Fy;
    S[6] = -7.0 / 3.0 * RHO0 * Fy;
    S[7] = RHO0 * Fz;
    S[8] = -7.0 / 3.0 * RHO0 * Fz;
    S[9] = 2.0 * RHO0 * (2.0 * ux * Fx - uy * Fy - uz * Fz) / phi;
    S[10] = 2.0 * RHO0 * (uy * Fy - uz * Fz) / phi;
    S[11] = RHO0 * (ux * Fy + uy * Fx) / phi;
    S[12] = RHO0 * (uy * Fz + uz * Fy) / phi;
    S[13] = RHO0 * (ux * Fz + uz * Fx) / phi;
    S[14] = 0.0;
  }
  return REF_OK;
}

/* Eq. 42 */
int ref_geq(double T, const double* u, double sigma, double varpi, double* geq) {
  if (!u || !geq) return REF_ERR_INVALID_ARG;
  double w[7];
  ref_weights(7, varpi, w);
  const double csT2 = varpi / 3.0;
  for (int i = 0; i < 7; ++i) {
    double eu = evel(7, 0, i) * u[0] + evel(7, 1, i) * u[1] + evel(7, 2, i) * u[2];
    geq[i] = w[i] * T * (sigma + eu / csT2);
  }
  return REF_OK;
}

/* Eq. 37 */
int ref_neq(double T, const double* u, double sigma, double varpi, double* neq) {
  if (!u || !neq) return REF_ERR_INVALID_ARG;
  neq[0] = T * sigma;
  neq[1] = T * u[0];
  neq[2] = T * u[1];
  neq[3] = T * u[2];
  neq[4] = T * varpi * sigma;
  neq[5] = 0.0;
  neq[6] = 0.0;
  return REF_OK;
}

/* Eqs. 27-28 with the full sum over directions (R1); dt = 1 */
int ref_velocity(int q, const double* f, const double* G, double phi, double nu, double K,
                 double F_phi, double* u) {
  if ((q != 19 && q != 15) || !f || !G || !u || !(K > 0.0)) return REF_ERR_INVALID_ARG;
  double v[3];
  for (int a = 0; a < 3; ++a) {
    double s = 0.0;
    for (int i = 0; i < q; ++i) s += evel(q, a, i) * f[i];
    v[a] = s / RHO0 + 0.5 * phi * G[a];
  }
  const double l0 = 0.5 * (1.0 + phi * 0.5 * nu / K);
  const double l1 = phi * 0.5 * F_phi / sqrt(K);
  const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double den = l0 + sqrt(l0 * l0 + l1 * vn);
  for (int a = 0; a < 3; ++a) u[a] = v[a] / den;
  return REF_OK;
}

/* Eq. 4 */
int ref_total_force(const double* u, const double* G, double phi, double nu, double K,
                    double F_phi, double* F) {
  if (!u || !G || !F || !(K > 0.0)) return REF_ERR_INVALID_ARG;
  const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (int a = 0; a < 3; ++a)
    F[a] = -phi * nu / K * u[a] - phi * F_phi / sqrt(K) * un * u[a] + phi * G[a];
  return REF_OK;
}

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): one output from state s */
int ref_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

uint64_t ref_splitmix64(uint64_t s) {
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double ref_noise(uint64_t seed, uint64_t n, double amp) {
  double r = (double)(ref_splitmix64(seed ^ n) >> 11) * (1.0 / 9007199254740992.0);
  return amp * (2.0 * r - 1.0);
}

/* ---------------------------------------------------------------- lattice */

struct ref_lattice {
  ref_params p;
  ref_derived d;
  int q;
  long long n;          /* node count */
  int e[3][19];
  int opp[19];
  double w[19];
  double M[19 * 19];
  double Minv[19 * 19];
  double lam[19];        /* diagonal of Lambda (Eq. 22 / Eq. 16) */
  int e7[3][7];
  int opp7[7];
  double om[7];          /* omega_k of Eq. 42 */
  double Qd[7];          /* diagonal of Q (Eq. 38) */
  double *f, *g;         /* pre-collision state */
  double *fp, *gp;       /* post-collision */
  double *accel;         /* optional [3][n] */
  double *mac;           /* [4][n]: u and T of the last collision (outlet rule) */
  int64_t t;
};

void ref_default_params(ref_params* p) {
  memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 8;
  p->q = 19;
  p->porosity = 1.0;
  p->darcy = 1.0;
  p->rayleigh = 0.0;
  p->prandtl = 1.0;
  p->mach = 0.1;
  p->forchheimer = 1.0;
  p->sigma = 1.0;
  p->J = 1.0;
  p->Gamma = 1.0;
  p->varpi = 0.5;
  /* Sec. 4 defaults */
  p->s_rho = 1.0;
  p->s_j = 1.0;
  p->s_e = 1.1;
  p->s_eps = 1.1;
  p->s_q = 1.1;
  p->s_pi = 1.1;
  p->s_m = 1.2;
  p->zeta_T = 1.0;
  p->zeta_e = 1.2;
  p->zeta_nu = 1.2;
  p->gravity_axis = 2;
  p->length_axis = 0;
  p->delta_T = 1.0;
  p->init_axis = -1;
  for (int k = 0; k < 6; ++k) {
    p->face[k].flow = REF_FLOW_WALL;
    p->face[k].heat = REF_HEAT_ADIABATIC;
  }
}

static int derive(const ref_params* p, ref_derived* d) {
  const int dims[3] = {p->nx, p->ny, p->nz};
  if (p->length_axis < 0 || p->length_axis > 2) return REF_ERR_INVALID_ARG;
  const double L = (double)dims[p->length_axis]; /* R7 */
  const double csT2 = p->varpi / 3.0;
  double s_nu;
  if (p->s_nu_set > 0.0) {
    s_nu = p->s_nu_set;
  } else if (p->reynolds > 0.0) {
    /* Eq. 51 read as the inverse (R4): nu = u_c L / Re, nu_e = J nu = cs^2 (1/s_nu - 1/2) */
    const double nu = p->u_char * L / p->reynolds;
    s_nu = 1.0 / (0.5 + p->J * nu / CS2);
  } else {
    /* Eq. 56 */
    if (!(p->rayleigh > 0.0)) return REF_ERR_INVALID_ARG;
    s_nu = 1.0 / (0.5 + p->mach * p->J * L * sqrt(3.0 * p->prandtl) / sqrt(p->rayleigh));
  }
  double zeta_a;
  if (p->zeta_alpha_set > 0.0) {
    zeta_a = p->zeta_alpha_set;
  } else {
    /* Eq. 56 / Eq. 51 */
    zeta_a = 1.0 / (0.5 + p->Gamma * CS2 * (1.0 / s_nu - 0.5) /
                              (p->J * p->sigma * csT2 * p->prandtl));
  }
  d->L = L;
  d->s_nu = s_nu;
  d->zeta_alpha = zeta_a;
  d->nu_e = CS2 * (1.0 / s_nu - 0.5);          /* Eq. 32 */
  d->nu = d->nu_e / p->J;                        /* Eq. 7, J = nu_e / nu */
  d->alpha_e = p->sigma * csT2 * (1.0 / zeta_a - 0.5); /* Eq. 41 */
  d->alpha = d->alpha_e / p->Gamma;              /* Eq. 7, Gamma = alpha_e / alpha */
  d->K = p->darcy * L * L;                       /* Eq. 7 */
  d->F_phi = p->forchheimer * 1.75 / sqrt(150.0 * p->porosity * p->porosity * p->porosity); /* Eq. 6 */
  d->gbeta = p->rayleigh * d->nu * d->alpha / (L * L * L) / p->delta_T; /* Eq. 7 */
  d->l0 = 0.5 * (1.0 + p->porosity * 0.5 * d->nu / d->K); /* Eq. 28 */
  d->l1 = p->porosity * 0.5 * d->F_phi / sqrt(d->K);
  return REF_OK;
}

static int check_params(const ref_params* p) {
  if (p->q != 19 && p->q != 15) return REF_ERR_INVALID_ARG;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return REF_ERR_INVALID_ARG;
  if (!(p->porosity > 0.0 && p->porosity <= 1.0)) return REF_ERR_INVALID_ARG;
  if (!(p->darcy > 0.0) || !(p->prandtl > 0.0) || !(p->delta_T > 0.0)) return REF_ERR_INVALID_ARG;
  if (!(p->rayleigh >= 0.0) || !(p->sigma > 0.0) || !(p->J > 0.0) || !(p->Gamma > 0.0))
    return REF_ERR_INVALID_ARG;
  if (!(p->varpi > 0.0 && p->varpi < 1.0)) return REF_ERR_INVALID_ARG;
  if (p->gravity_axis < 0 || p->gravity_axis > 2) return REF_ERR_INVALID_ARG;
  if (p->init_axis < -1 || p->init_axis > 2) return REF_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a) {
    const ref_face* lo = &p->face[2 * a];
    const ref_face* hi = &p->face[2 * a + 1];
    int per_lo = lo->flow == REF_FLOW_PERIODIC, per_hi = hi->flow == REF_FLOW_PERIODIC;
    if (per_lo != per_hi) return REF_ERR_INVALID_ARG;
    if ((lo->heat == REF_HEAT_PERIODIC) != per_lo || (hi->heat == REF_HEAT_PERIODIC) != per_hi)
      return REF_ERR_INVALID_ARG;
    for (int s = 0; s < 2; ++s) {
      const ref_face* fc = &p->face[2 * a + s];
      if (fc->flow != REF_FLOW_PERIODIC && fc->flow != REF_FLOW_WALL && fc->flow != REF_FLOW_OUTLET)
        return REF_ERR_UNSUPPORTED;
      if (fc->heat != REF_HEAT_PERIODIC && fc->heat != REF_HEAT_ADIABATIC &&
          fc->heat != REF_HEAT_ISOTHERMAL && fc->heat != REF_HEAT_OUTFLOW)
        return REF_ERR_UNSUPPORTED;
    }
  }
  return REF_OK;
}

static void node_xyz(const ref_lattice* h, long long n, int* x, int* y, int* z) {
  *x = (int)(n % h->p.nx);
  *y = (int)((n / h->p.nx) % h->p.ny);
  *z = (int)(n / ((long long)h->p.nx * h->p.ny));
}

int ref_create(const ref_params* p, ref_lattice** out) {
  if (!p || !out) return REF_ERR_INVALID_ARG;
  *out = NULL;
  int st = check_params(p);
  if (st != REF_OK) return st;
  ref_derived d;
  st = derive(p, &d);
  if (st != REF_OK) return st;
  if (!(d.s_nu > 0.0 && d.s_nu < 2.0) || !(d.zeta_alpha > 0.0 && d.zeta_alpha < 2.0))
    return REF_ERR_INVALID_ARG;

  ref_lattice* h = (ref_lattice*)calloc(1, sizeof(ref_lattice));
  if (!h) return REF_ERR_OUT_OF_MEMORY;
  h->p = *p;
  h->d = d;
  h->q = p->q;
  h->n = (long long)p->nx * p->ny * p->nz;
  const int q = h->q;
  for (int a = 0; a < 3; ++a) {
    for (int i = 0; i < q; ++i) h->e[a][i] = evel(q, a, i);
    for (int i = 0; i < 7; ++i) h->e7[a][i] = evel(7, a, i);
  }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j)
      if (h->e[0][j] == -h->e[0][i] && h->e[1][j] == -h->e[1][i] && h->e[2][j] == -h->e[2][i])
        h->opp[i] = j;
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j)
      if (h->e7[0][j] == -h->e7[0][i] && h->e7[1][j] == -h->e7[1][i] &&
          h->e7[2][j] == -h->e7[2][i])
        h->opp7[i] = j;
  ref_weights(q, p->varpi, h->w);
  ref_weights(7, p->varpi, h->om);
  ref_matrix(q, h->M);
  if (ref_matrix_inverse(q, h->Minv) != REF_OK) {
    free(h);
    return REF_ERR_INVALID_ARG;
  }
  if (q == 19) {
    /* Eq. 22 */
    const double lam[19] = {p->s_rho, p->s_e,  p->s_eps, p->s_j, p->s_q,  p->s_j,  p->s_q,
                            p->s_j,   p->s_q,  d.s_nu,   p->s_pi, d.s_nu, p->s_pi, d.s_nu,
                            d.s_nu,   d.s_nu,  p->s_m,   p->s_m, p->s_m};
    memcpy(h->lam, lam, sizeof(lam));
  } else {
    /* Eq. 16 */
    const double lam[15] = {p->s_rho, p->s_e, p->s_eps, p->s_j, p->s_q, p->s_j, p->s_q, p->s_j,
                            p->s_q,   d.s_nu, d.s_nu,   d.s_nu, d.s_nu, d.s_nu, p->s_m};
    memcpy(h->lam, lam, sizeof(lam));
  }
  /* Eq. 38 */
  const double Qd[7] = {p->zeta_T, d.zeta_alpha, d.zeta_alpha, d.zeta_alpha,
                        p->zeta_e, p->zeta_nu,   p->zeta_nu};
  memcpy(h->Qd, Qd, sizeof(Qd));

  const size_t N = (size_t)h->n;
  h->f = (double*)malloc(sizeof(double) * N * q);
  h->fp = (double*)malloc(sizeof(double) * N * q);
  h->g = (double*)malloc(sizeof(double) * N * 7);
  h->gp = (double*)malloc(sizeof(double) * N * 7);
  h->mac = (double*)malloc(sizeof(double) * N * 4);
  if (!h->f || !h->fp || !h->g || !h->gp || !h->mac) {
    ref_destroy(h);
    return REF_ERR_OUT_OF_MEMORY;
  }

  /* initial state: f = f^eq(rho0, u0) (Eq. 24 / Eq. 18), g = g^eq(T, u0) (Eq. 42) */
  const int dims[3] = {p->nx, p->ny, p->nz};
  const double* u0 = p->init_u;
  double feq[19];
  ref_feq(q, RHO0, u0, p->porosity, feq);
  for (long long n = 0; n < h->n; ++n) {
    int c[3];
    node_xyz(h, n, &c[0], &c[1], &c[2]);
    double T = p->T_ref;
    if (p->init_axis >= 0) {
      const double s = ((double)c[p->init_axis] + 0.5) / (double)dims[p->init_axis];
      T = p->init_T_lo + (p->init_T_hi - p->init_T_lo) * s;
    }
    const double noise = ref_noise(p->seed, (uint64_t)n, p->noise_amp);
    T = T + noise;
    double geq[7];
    ref_geq(T, u0, p->sigma, p->varpi, geq);
    for (int i = 0; i < q; ++i) h->f[(size_t)i * N + n] = feq[i];
    for (int k = 0; k < 7; ++k) h->g[(size_t)k * N + n] = geq[k];
  }
  h->t = 0;
  *out = h;
  return REF_OK;
}

void ref_destroy(ref_lattice* h) {
  if (!h) return;
  free(h->f);
  free(h->fp);
  free(h->g);
  free(h->gp);
  free(h->accel);
  free(h->mac);
  free(h);
}

int ref_get_derived(const ref_lattice* h, ref_derived* d) {
  if (!h || !d) return REF_ERR_INVALID_ARG;
  *d = h->d;
  return REF_OK;
}

int64_t ref_time(const ref_lattice* h) { return h ? h->t : -1; }

int ref_set_accel_field(ref_lattice* h, const double* a) {
  if (!h) return REF_ERR_INVALID_ARG;
  free(h->accel);
  h->accel = NULL;
  if (!a) return REF_OK;
  h->accel = (double*)malloc(sizeof(double) * 3 * (size_t)h->n);
  if (!h->accel) return REF_ERR_OUT_OF_MEMORY;
  memcpy(h->accel, a, sizeof(double) * 3 * (size_t)h->n);
  return REF_OK;
}

/* G of Eq. 5 at node n for temperature T (R6) */
static void buoyancy(const ref_lattice* h, long long n, double T, double G[3]) {
  for (int a = 0; a < 3; ++a) G[a] = h->p.accel[a];
  G[h->p.gravity_axis] += h->d.gbeta * (T - h->p.T_ref);
  if (h->accel && n >= 0)
    for (int a = 0; a < 3; ++a) G[a] += h->accel[(size_t)a * h->n + n];
}

/* macroscopic state of one node's pre-collision populations */
static void node_macro(const ref_lattice* h, long long n, const double* f, const double* g,
                       double* rho, double u[3], double* T, double G[3], double F[3]) {
  const int q = h->q;
  double r = 0.0;
  for (int i = 0; i < q; ++i) r += f[i]; /* Eq. 25 */
  double n0 = 0.0;
  for (int k = 0; k < 7; ++k) n0 += g[k];
  const double temp = n0 / h->p.sigma; /* Eq. 39 */
  buoyancy(h, n, temp, G);
  ref_velocity(q, f, G, h->p.porosity, h->d.nu, h->d.K, h->d.F_phi, u);
  ref_total_force(u, G, h->p.porosity, h->d.nu, h->d.K, h->d.F_phi, F);
  *rho = r;
  *T = temp;
}

static void collide(const ref_lattice* h, long long n, const double* f, const double* g,
                    double* fo, double* go, double* rho_o, double* u_o, double* T_o,
                    double* F_o) {
  const int q = h->q;
  const double phi = h->p.porosity;
  double rho, u[3], T, G[3], F[3];
  node_macro(h, n, f, g, &rho, u, &T, G, F);

  /* flow: Eqs. 9-11 */
  double m[19], meq[19], S[19], ms[19];
  for (int k = 0; k < q; ++k) {
    double s = 0.0;
    for (int i = 0; i < q; ++i) s += h->M[k * q + i] * f[i];
    m[k] = s;
  }
  ref_meq(q, rho, u, phi, meq);
  ref_forcing_moments(q, u, F, phi, S);
  for (int k = 0; k < q; ++k)
    ms[k] = m[k] - h->lam[k] * (m[k] - meq[k]) + (1.0 - 0.5 * h->lam[k]) * S[k];
  for (int i = 0; i < q; ++i) {
    double s = 0.0;
    for (int k = 0; k < q; ++k) s += h->Minv[i * q + k] * ms[k];
    fo[i] = s;
  }

  /* temperature: Eqs. 34, 36-38, 43 */
  double nm[7], neq[7], ns[7];
  for (int k = 0; k < 7; ++k) {
    double s = 0.0;
    for (int i = 0; i < 7; ++i) s += N7[k][i] * g[i];
    nm[k] = s;
  }
  ref_neq(T, u, h->p.sigma, h->p.varpi, neq);
  for (int k = 0; k < 7; ++k) ns[k] = nm[k] - h->Qd[k] * (nm[k] - neq[k]);
  for (int i = 0; i < 7; ++i) {
    double s = 0.0;
    for (int k = 0; k < 7; ++k) s += N7INV[i][k] * ns[k];
    go[i] = s;
  }
  if (rho_o) *rho_o = rho;
  if (u_o) memcpy(u_o, u, sizeof(u));
  if (T_o) *T_o = T;
  if (F_o) memcpy(F_o, F, sizeof(F));
}

int ref_collide_node(const ref_lattice* h, const double* f, const double* g, double* fo,
                     double* go, double* rho, double* u, double* T, double* F) {
  if (!h || !f || !g || !fo || !go) return REF_ERR_INVALID_ARG;
  collide(h, -1, f, g, fo, go, rho, u, T, F);
  return REF_OK;
}

/* Destination of a link from node (x,y,z) along e: returns 1 and the
 * destination index if the link stays in the box (periodic faces wrap),
 * otherwise 0 and the face whose rule applies: the first wall face crossed in
 * face order, else the first outlet face crossed (R5). */
static int link_target(const ref_lattice* h, const int c[3], const int e[3], long long* dst,
                       int* face) {
  const int dims[3] = {h->p.nx, h->p.ny, h->p.nz};
  int d[3];
  int hit = -1, outlet = -1;
  for (int a = 0; a < 3; ++a) {
    d[a] = c[a] + e[a];
    if (d[a] < 0 || d[a] >= dims[a]) {
      const int fc = 2 * a + (d[a] < 0 ? 0 : 1);
      if (h->p.face[fc].flow == REF_FLOW_PERIODIC) {
        d[a] = (d[a] + dims[a]) % dims[a];
      } else if (h->p.face[fc].flow == REF_FLOW_OUTLET) {
        if (outlet < 0) outlet = fc;
      } else if (hit < 0) {
        hit = fc;
      }
    }
  }
  if (hit < 0) hit = outlet;
  if (hit >= 0) {
    *face = hit;
    return 0;
  }
  *dst = d[0] + (long long)dims[0] * (d[1] + (long long)dims[1] * d[2]);
  return 1;
}

int ref_step(ref_lattice* h, int64_t nsteps) {
  if (!h || nsteps < 0) return REF_ERR_INVALID_ARG;
  const int q = h->q;
  const long long N = h->n;
  for (int64_t s = 0; s < nsteps; ++s) {
    /* collide every node */
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < N; ++n) {
      double f[19], g[7], fo[19], go[7], u[3], T;
      for (int i = 0; i < q; ++i) f[i] = h->f[(size_t)i * N + n];
      for (int k = 0; k < 7; ++k) g[k] = h->g[(size_t)k * N + n];
      collide(h, n, f, g, fo, go, NULL, u, &T, NULL);
      for (int a = 0; a < 3; ++a) h->mac[(size_t)a * N + n] = u[a];
      h->mac[(size_t)3 * N + n] = T;
      for (int i = 0; i < q; ++i) h->fp[(size_t)i * N + n] = fo[i];
      for (int k = 0; k < 7; ++k) h->gp[(size_t)k * N + n] = go[k];
    }
    /* stream every post-collision population (Eqs. 10, 35) */
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < N; ++n) {
      int c[3];
      node_xyz(h, n, &c[0], &c[1], &c[2]);
      for (int i = 0; i < q; ++i) {
        const int e[3] = {h->e[0][i], h->e[1][i], h->e[2][i]};
        long long dst;
        int face;
        const double v = h->fp[(size_t)i * N + n];
        if (link_target(h, c, e, &dst, &face)) {
          h->f[(size_t)i * N + dst] = v;
        } else if (h->p.face[face].flow == REF_FLOW_OUTLET) {
          /* open boundary at rho0 (R5) */
          const int o = h->opp[i];
          const double u[3] = {h->mac[n], h->mac[(size_t)N + n], h->mac[(size_t)2 * N + n]};
          const double eu = h->e[0][o] * u[0] + h->e[1][o] * u[1] + h->e[2][o] * u[2];
          const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
          const double phi = h->p.porosity;
          const double even = h->w[o] * RHO0 * (1.0 + eu * eu / (2.0 * phi * CS2 * CS2) - uu / (2.0 * phi * CS2));
          h->f[(size_t)o * N + n] = -v + 2.0 * even;
        } else {
          /* bounce back into this node along the opposite direction (R5) */
          const int o = h->opp[i];
          const double* uw = h->p.face[face].u_wall;
          const double eu = h->e[0][o] * uw[0] + h->e[1][o] * uw[1] + h->e[2][o] * uw[2];
          h->f[(size_t)o * N + n] = v + 2.0 * h->w[o] * RHO0 * eu / CS2;
        }
      }
      for (int k = 0; k < 7; ++k) {
        const int e[3] = {h->e7[0][k], h->e7[1][k], h->e7[2][k]};
        long long dst;
        int face;
        const double v = h->gp[(size_t)k * N + n];
        if (link_target(h, c, e, &dst, &face)) {
          h->g[(size_t)k * N + dst] = v;
        } else {
          const int o = h->opp7[k];
          if (h->p.face[face].heat == REF_HEAT_ISOTHERMAL)
            h->g[(size_t)o * N + n] = -v + 2.0 * h->om[o] * h->p.sigma * h->p.face[face].T_wall;
          else if (h->p.face[face].heat == REF_HEAT_OUTFLOW)
            h->g[(size_t)o * N + n] = -v + 2.0 * h->om[o] * h->p.sigma * h->mac[(size_t)3 * N + n];
          else
            h->g[(size_t)o * N + n] = v;
        }
      }
    }
    h->t += 1;
  }
  return REF_OK;
}

int ref_fields(const ref_lattice* h, double* rho, double* ux, double* uy, double* uz,
               double* T) {
  if (!h) return REF_ERR_INVALID_ARG;
  const int q = h->q;
  const long long N = h->n;
  for (long long n = 0; n < N; ++n) {
    double f[19], g[7], r, u[3], t, G[3], F[3];
    for (int i = 0; i < q; ++i) f[i] = h->f[(size_t)i * N + n];
    for (int k = 0; k < 7; ++k) g[k] = h->g[(size_t)k * N + n];
    node_macro(h, n, f, g, &r, u, &t, G, F);
    if (rho) rho[n] = r;
    if (ux) ux[n] = u[0];
    if (uy) uy[n] = u[1];
    if (uz) uz[n] = u[2];
    if (T) T[n] = t;
  }
  return REF_OK;
}

/* Heat entering the fluid through an isothermal face during the last
 * streaming: at a wall node the incoming population k was set by
 * anti-bounce-back from the outgoing one, g_k = -g*_kbar + 2 omega_k sigma T_w,
 * so the net flux g_k - g*_kbar equals 2 g_k - 2 omega_k sigma T_w.  The face
 * average, scaled by L / (alpha_e delta_T), is the face Nusselt number of
 * Eqs. 53-55 (midpoint rule over the face). */
int ref_nusselt(const ref_lattice* h, double nu[6]) {
  if (!h || !nu) return REF_ERR_INVALID_ARG;
  const int dims[3] = {h->p.nx, h->p.ny, h->p.nz};
  const long long N = h->n;
  for (int fc = 0; fc < 6; ++fc) {
    nu[fc] = 0.0;
    if (h->p.face[fc].heat != REF_HEAT_ISOTHERMAL) continue;
    const int a = fc / 2, side = fc % 2;
    /* direction pointing from the wall into the fluid */
    int kin = -1;
    for (int k = 1; k < 7; ++k) {
      if (h->e7[a][k] == (side == 0 ? 1 : -1)) kin = k;
    }
    const double Tw = h->p.face[fc].T_wall;
    double sum = 0.0;
    long long count = 0;
    for (long long n = 0; n < N; ++n) {
      int c[3];
      node_xyz(h, n, &c[0], &c[1], &c[2]);
      if (c[a] != (side == 0 ? 0 : dims[a] - 1)) continue;
      const double gk = h->g[(size_t)kin * N + n];
      sum += 2.0 * gk - 2.0 * h->om[kin] * h->p.sigma * Tw;
      count += 1;
    }
    nu[fc] = (sum / (double)count) * h->d.L / (h->d.alpha_e * h->p.delta_T);
  }
  return REF_OK;
}

int ref_get_state(const ref_lattice* h, double* f, double* g) {
  if (!h) return REF_ERR_INVALID_ARG;
  if (f) memcpy(f, h->f, sizeof(double) * (size_t)h->n * h->q);
  if (g) memcpy(g, h->g, sizeof(double) * (size_t)h->n * 7);
  return REF_OK;
}

int ref_set_state(ref_lattice* h, const double* f, const double* g) {
  if (!h) return REF_ERR_INVALID_ARG;
  if (f) memcpy(h->f, f, sizeof(double) * (size_t)h->n * h->q);
  if (g) memcpy(h->g, g, sizeof(double) * (size_t)h->n * 7);
  return REF_OK;
}
