/*
 * enthalpy_oracle.c -- FP64 CPU oracle of the enthalpy-based D3Q7-MRT model
 * for solid-liquid phase change (Liu & He, arXiv:1611.03329, App. B,
 * Eqs. B4-B13), in the conduction setting of the paper's melting test
 * (Sec. 4.3: the velocity is zero throughout).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, never by the product library,
 * and sharing no code with it.
 *
 * One step, for every node: effective enthalpy En = sum g (Eq. B7); T and the
 * liquid fraction f_l from En (Eqs. B8, B9); moments n = N g (Eq. 36); the
 * equilibrium moments of Eq. B6 with u = 0; the relaxation n* = n - Q(n - n^eq)
 * (Eq. 34) with zeta_alpha from the local diffusivity alpha_l f_l +
 * alpha_s (1 - f_l) (Eq. B11, Sec. 4.3); g* = N^-1 n* (Eq. 43); then streaming
 * along the D3Q7 links with the wall rules below.
 *
 * Readings (where the paper is silent):
 *   E1  heat capacity ratios of Eq. B4 with rho_l = rho_s = rho0 and the matrix
 *       given as r_m = rho_m c_pm / (rho_l c_pl): sigma_l = phi + (1-phi) r_m,
 *       sigma_s = phi c_ps/c_pl + (1-phi) r_m.
 *   E2  c_p,ref = 2/(1/c_pl + 1/c_ps), the first form of Eq. B13.
 *   E3  the liquidus enthalpy is En_l = sigma_l c_pl T_l + phi L_a (the text of
 *       Eq. B8 with f_l = 1).
 *   E4  walls: halfway anti-bounce-back at a wall temperature T_w with the
 *       moving-population equilibrium of Eq. B12 at u = 0,
 *       g_kbar = -g*_k + 2 (varpi/6) c_p,ref T_w; adiabatic walls bounce back;
 *       periodic faces wrap.
 *   E5  initial state: uniform T_init, En from Eqs. B8-B9 inverted, g = g^eq
 *       of Eq. B12 at u = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

/* D3Q7 velocities (the first seven of Eq. 12) */
static const int E7[3][7] = {{0, 1, -1, 0, 0, 0, 0}, {0, 0, 0, 1, -1, 0, 0}, {0, 0, 0, 0, 0, 1, -1}};
static const int OPP7[7] = {0, 2, 1, 4, 3, 6, 5};

/* Eq. 36 */
static const double N7E[7][7] = {
    {1, 1, 1, 1, 1, 1, 1},   {0, 1, -1, 0, 0, 0, 0},  {0, 0, 0, 1, -1, 0, 0},  {0, 0, 0, 0, 0, 1, -1},
    {0, 1, 1, 1, 1, 1, 1},   {0, 1, 1, -1, -1, 0, 0}, {0, 1, 1, 0, 0, -1, -1}};
/* Eq. 43 */
static const double N7EINV[7][7] = {
    {1, 0, 0, 0, -1, 0, 0},
    {0, 0.5, 0, 0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0},
    {0, -0.5, 0, 0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0},
    {0, 0, 0.5, 0, 1.0 / 6.0, -1.0 / 3.0, 1.0 / 6.0},
    {0, 0, -0.5, 0, 1.0 / 6.0, -1.0 / 3.0, 1.0 / 6.0},
    {0, 0, 0, 0.5, 1.0 / 6.0, 1.0 / 6.0, -1.0 / 3.0},
    {0, 0, 0, -0.5, 1.0 / 6.0, 1.0 / 6.0, -1.0 / 3.0}};

struct ref_enthalpy {
  ref_enthalpy_params p;
  long long n;
  double *g, *gn; /* [7][n] */
  int64_t t;
  double sigma_l, sigma_s, cpref, En_s, En_l, csT2;
};

static void phase(const ref_enthalpy* h, double En, double* T, double* fl) {
  const ref_enthalpy_params* p = &h->p;
  if (En <= h->En_s) {                             /* Eq. B8, B9: solid */
    *T = En / (h->sigma_s * p->c_pl);
    *fl = 0.0;
  } else if (En >= h->En_l) {                      /* liquid */
    *T = p->T_liquidus + (En - h->En_l) / (h->sigma_l * p->c_pl);
    *fl = 1.0;
  } else {                                         /* mushy */
    const double s = (En - h->En_s) / (h->En_l - h->En_s);
    *T = p->T_solidus + s * (p->T_liquidus - p->T_solidus);
    *fl = s;
  }
}

static double enthalpy_of(const ref_enthalpy* h, double T) {
  const ref_enthalpy_params* p = &h->p;
  if (T <= p->T_solidus) return h->sigma_s * p->c_pl * T;
  if (T >= p->T_liquidus) return h->En_l + h->sigma_l * p->c_pl * (T - p->T_liquidus);
  /* inside the mushy range the map is not one-to-one for T_s = T_l; take the solid side */
  return h->En_s + (T - p->T_solidus) / (p->T_liquidus - p->T_solidus) * (h->En_l - h->En_s);
}

int ref_enthalpy_create(const ref_enthalpy_params* p, ref_enthalpy** out) {
  if (!p || !out) return REF_ERR_INVALID_ARG;
  *out = NULL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->varpi > 0.0 && p->varpi < 1.0) ||
      !(p->porosity > 0.0 && p->porosity <= 1.0) || !(p->c_pl > 0.0) || !(p->c_ps > 0.0) ||
      !(p->latent >= 0.0) || !(p->T_liquidus >= p->T_solidus) || !(p->alpha_l > 0.0) || !(p->alpha_s > 0.0))
    return REF_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a)
    if ((p->heat[2 * a] == 0) != (p->heat[2 * a + 1] == 0)) return REF_ERR_INVALID_ARG;
  ref_enthalpy* h = (ref_enthalpy*)calloc(1, sizeof(ref_enthalpy));
  if (!h) return REF_ERR_OUT_OF_MEMORY;
  h->p = *p;
  h->n = (long long)p->nx * p->ny * p->nz;
  h->g = (double*)malloc(sizeof(double) * 7 * (size_t)h->n);
  h->gn = (double*)malloc(sizeof(double) * 7 * (size_t)h->n);
  if (!h->g || !h->gn) {
    ref_enthalpy_destroy(h);
    return REF_ERR_OUT_OF_MEMORY;
  }
  h->sigma_l = p->porosity + (1.0 - p->porosity) * p->matrix_heat;                       /* E1 */
  h->sigma_s = p->porosity * p->c_ps / p->c_pl + (1.0 - p->porosity) * p->matrix_heat;
  h->cpref = 2.0 / (1.0 / p->c_pl + 1.0 / p->c_ps);                                      /* E2 */
  h->En_s = h->sigma_s * p->c_pl * p->T_solidus;
  h->En_l = h->sigma_l * p->c_pl * p->T_liquidus + p->porosity * p->latent;              /* E3 */
  h->csT2 = p->varpi / 3.0;
  const double En = enthalpy_of(h, p->T_init);                                           /* E5 */
  double T, fl;
  phase(h, En, &T, &fl);
  const long long N = h->n;
  for (long long n = 0; n < N; ++n) {
    h->g[n] = En - p->varpi * h->cpref * T;                                              /* Eq. B12 */
    for (int k = 1; k < 7; ++k) h->g[(size_t)k * N + n] = p->varpi * h->cpref * T / 6.0;
  }
  *out = h;
  return REF_OK;
}

void ref_enthalpy_destroy(ref_enthalpy* h) {
  if (!h) return;
  free(h->g);
  free(h->gn);
  free(h);
}

int64_t ref_enthalpy_time(const ref_enthalpy* h) { return h ? h->t : -1; }

/* collision at one node: g[7] -> gs[7] */
static void collide(const ref_enthalpy* h, const double* g, double* gs) {
  const ref_enthalpy_params* p = &h->p;
  double En = 0.0;
  for (int k = 0; k < 7; ++k) En += g[k];                                                /* Eq. B7 */
  double T, fl;
  phase(h, En, &T, &fl);
  const double alpha = p->alpha_l * fl + p->alpha_s * (1.0 - fl);
  const double za = 1.0 / (0.5 + alpha / h->csT2);                                      /* Eq. B11 */
  double m[7], neq[7] = {En, 0.0, 0.0, 0.0, p->varpi * h->cpref * T, 0.0, 0.0};        /* Eq. B6, u = 0 */
  const double Q[7] = {1.0, za, za, za, p->zeta_e, p->zeta_nu, p->zeta_nu};            /* Eq. 38 */
  for (int r = 0; r < 7; ++r) {
    m[r] = 0.0;
    for (int k = 0; k < 7; ++k) m[r] += N7E[r][k] * g[k];
  }
  for (int r = 0; r < 7; ++r) m[r] -= Q[r] * (m[r] - neq[r]);
  for (int k = 0; k < 7; ++k) {
    gs[k] = 0.0;
    for (int r = 0; r < 7; ++r) gs[k] += N7EINV[k][r] * m[r];
  }
}

int ref_enthalpy_step(ref_enthalpy* h, int64_t nsteps) {
  if (!h || nsteps < 0) return REF_ERR_INVALID_ARG;
  const ref_enthalpy_params* p = &h->p;
  const long long N = h->n;
  const int dims[3] = {p->nx, p->ny, p->nz};
  for (int64_t s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < N; ++n) {
      double g[7], gs[7];
      for (int k = 0; k < 7; ++k) g[k] = h->g[(size_t)k * N + n];
      collide(h, g, gs);
      const int c[3] = {(int)(n % p->nx), (int)((n / p->nx) % p->ny), (int)(n / ((long long)p->nx * p->ny))};
      h->gn[n] = gs[0];
      for (int k = 1; k < 7; ++k) {
        int d[3], wall_face = -1;
        for (int a = 0; a < 3; ++a) {
          d[a] = c[a] + E7[a][k];
          if (d[a] < 0 || d[a] >= dims[a]) {
            const int f = 2 * a + (d[a] < 0 ? 0 : 1);
            if (p->heat[f] == 0) d[a] = (d[a] + dims[a]) % dims[a];   /* periodic */
            else wall_face = f;
          }
        }
        if (wall_face < 0) {
          const long long dn = d[0] + (long long)p->nx * (d[1] + (long long)p->ny * d[2]);
          h->gn[(size_t)k * N + dn] = gs[k];
        } else {                                                    /* E4 */
          const int kb = OPP7[k];
          double v = gs[k];
          if (p->heat[wall_face] == 2) v = -gs[k] + 2.0 * (p->varpi / 6.0) * h->cpref * p->T_wall[wall_face];
          h->gn[(size_t)kb * N + n] = v;
        }
      }
    }
    double* tmp = h->g;
    h->g = h->gn;
    h->gn = tmp;
    h->t += 1;
  }
  return REF_OK;
}

int ref_enthalpy_fields(const ref_enthalpy* h, double* T, double* En, double* fl) {
  if (!h) return REF_ERR_INVALID_ARG;
  const long long N = h->n;
  for (long long n = 0; n < N; ++n) {
    double e = 0.0;
    for (int k = 0; k < 7; ++k) e += h->g[(size_t)k * N + n];
    double t, f;
    phase(h, e, &t, &f);
    if (T) T[n] = t;
    if (En) En[n] = e;
    if (fl) fl[n] = f;
  }
  return REF_OK;
}

int ref_enthalpy_get_state(const ref_enthalpy* h, double* g) {
  if (!h || !g) return REF_ERR_INVALID_ARG;
  memcpy(g, h->g, sizeof(double) * 7 * (size_t)h->n);
  return REF_OK;
}

int ref_enthalpy_set_state(ref_enthalpy* h, const double* g) {
  if (!h || !g) return REF_ERR_INVALID_ARG;
  memcpy(h->g, g, sizeof(double) * 7 * (size_t)h->n);
  return REF_OK;
}

int ref_enthalpy_phase(const ref_enthalpy* h, double En, double* T, double* fl) {
  if (!h || !T || !fl) return REF_ERR_INVALID_ARG;
  phase(h, En, T, fl);
  return REF_OK;
}
