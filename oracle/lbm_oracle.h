/*
 * lbm_oracle.h -- plain FP64 CPU oracle for the REV-scale double-distribution-
 * function MRT lattice Boltzmann model of Liu & He, "Three-dimensional
 * multiple-relaxation-time lattice Boltzmann model for convection heat transfer
 * in porous media at the REV scale" (arXiv:1611.03329).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the GPU path can be
 * checked against something written directly from the paper.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it;
 * the product library never calls it and shares no source with it.
 *
 * Conventions (fixed here, stated once):
 *   - lattice units rho0 = dt = dx = c = 1 (Sec. 4 defaults), cs^2 = 1/3,
 *     csT^2 = varpi/3 (Eq. 40);
 *   - node (x,y,z), 0 <= x < nx ..., linear index n = x + nx*(y + ny*z);
 *     non-periodic faces are halfway walls at -1/2 and n-1/2;
 *   - population arrays are [q][z][y][x] (population-major), FP64;
 *   - the state at integer time t is the PRE-collision populations f(t), g(t);
 *     one step is "collide every node (Eqs. 9, 34) then stream (Eqs. 10, 35)
 *     with the wall rules applied to links that leave the box";
 *   - all fields and diagnostics at time t are computed from that state.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define REF_OK 0
#define REF_ERR_INVALID_ARG 1
#define REF_ERR_OUT_OF_MEMORY 2
#define REF_ERR_UNSUPPORTED 5

/* flow rule of a face */
#define REF_FLOW_PERIODIC 0
#define REF_FLOW_WALL 1      /* halfway bounce-back; u_wall adds the moving-wall term */
#define REF_FLOW_OUTLET 3    /* open boundary at rho0: anti-bounce-back to the even part
                                of f^eq(rho0, u) with u the node's own velocity */
/* thermal rule of a face */
#define REF_HEAT_PERIODIC 0
#define REF_HEAT_ADIABATIC 1   /* bounce-back of g: zero normal flux */
#define REF_HEAT_ISOTHERMAL 2  /* anti-bounce-back of g to T_wall */
#define REF_HEAT_OUTFLOW 3     /* anti-bounce-back to the node's own temperature */

typedef struct {
  int32_t flow;
  int32_t heat;
  double T_wall;
  double u_wall[3];
} ref_face;

/* Face order: 0 = -x, 1 = +x, 2 = -y, 3 = +y, 4 = -z, 5 = +z. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t q;               /* 19 (D3Q19, Sec. 3.1.2) or 15 (D3Q15, Sec. 3.1.1) */
  double porosity;         /* phi in (0,1] */
  double darcy;            /* Da = K/L^2 > 0 (Eq. 7) */
  double rayleigh;         /* Ra >= 0 (Eq. 7) */
  double prandtl;          /* Pr > 0 (Eq. 7) */
  double reynolds;         /* > 0 selects the channel mapping (Eq. 51) */
  double u_char;           /* channel characteristic speed (Re = L u_c / nu) */
  double mach;             /* cavity mapping (Eq. 56), Ma = u_c / cs */
  double forchheimer;      /* multiplier on Eq. 6's F_phi: 1 = generalized non-Darcy, 0 = Brinkman */
  double sigma, J, Gamma, varpi;
  double s_rho, s_e, s_eps, s_j, s_q, s_pi, s_m;  /* flow rates (Eqs. 16, 22) */
  double zeta_T, zeta_e, zeta_nu;                 /* thermal rates (Eq. 38) */
  double s_nu_set;         /* > 0: use this s_nu instead of Eq. 56 / Eq. 51 */
  double zeta_alpha_set;   /* > 0: use this zeta_alpha instead of Eq. 56 / Eq. 51 */
  int32_t gravity_axis;    /* axis along which buoyancy acts (0,1,2) */
  int32_t length_axis;     /* axis whose node count is the characteristic length L */
  double T_ref;            /* T0 of Eq. 5 */
  double delta_T;          /* temperature scale in Ra (Eq. 7); > 0 */
  double accel[3];         /* constant external acceleration a of Eq. 5 */
  ref_face face[6];
  int32_t init_axis;       /* -1: uniform T_ref; else linear in that axis ... */
  double init_T_lo;        /* ... from init_T_lo at the -1/2 face ... */
  double init_T_hi;        /* ... to init_T_hi at the n-1/2 face */
  uint64_t seed;
  double noise_amp;        /* T += noise_amp*(2r-1), r from SplitMix64(seed ^ n) */
  double init_u[3];        /* initial velocity: f = f^eq(rho0, init_u), g = g^eq(T, init_u) */
} ref_params;

typedef struct {
  double L, s_nu, zeta_alpha, nu_e, nu, alpha_e, alpha, K, F_phi, gbeta, l0, l1;
} ref_derived;

typedef struct ref_lattice ref_lattice;

void ref_default_params(ref_params* p);
int ref_create(const ref_params* p, ref_lattice** out);
void ref_destroy(ref_lattice* h);
int ref_get_derived(const ref_lattice* h, ref_derived* d);
int ref_step(ref_lattice* h, int64_t nsteps);
int64_t ref_time(const ref_lattice* h);
/* rho, ux, uy, uz, T at the current time; any pointer may be NULL */
int ref_fields(const ref_lattice* h, double* rho, double* ux, double* uy, double* uz, double* T);
/* per face: mean heat flux INTO the fluid over the face's nodes, times L/(alpha_e*delta_T);
 * 0 for faces that are not isothermal. */
int ref_nusselt(const ref_lattice* h, double nu[6]);
/* logical pre-collision state, [q][z][y][x] and [7][z][y][x] */
int ref_get_state(const ref_lattice* h, double* f, double* g);
int ref_set_state(ref_lattice* h, const double* f, const double* g);
/* optional per-node acceleration field, [3][z][y][x], added to a in Eq. 5; NULL clears */
int ref_set_accel_field(ref_lattice* h, const double* a);
/* one node's collision with the lattice's parameters: f[q], g[7] -> fo[q], go[7];
 * also returns rho, u[3], T, F[3] of the pre-collision state. */
int ref_collide_node(const ref_lattice* h, const double* f, const double* g,
                     double* fo, double* go, double* rho, double* u, double* T, double* F);

/* ---- pieces of the model, exposed for the unit pins ---- */
/* velocity set e[3][q] (Eq. 19 / Eq. 12; q = 7 gives the D3Q7 set) */
int ref_velocities(int q, int* e);
int ref_weights(int q, double varpi, double* w);
/* transformation matrix: M of Eq. A2 (q=19), Eq. A1 (q=15), N of Eq. 36 (q=7) */
int ref_matrix(int q, double* M);
/* inverse of that matrix (q=19, 15: by Gauss-Jordan elimination; q=7: Eq. 43) */
int ref_matrix_inverse(int q, double* Minv);
/* f^eq in velocity space (Eq. 24 / Eq. 18) */
int ref_feq(int q, double rho, const double* u, double phi, double* feq);
/* m^eq in moment space (Eq. 21 / Eq. 15; conserved rows rho, rho0*u) */
int ref_meq(int q, double rho, const double* u, double phi, double* meq);
/* forcing in moment space (Eq. 23 / Eq. 17) */
int ref_forcing_moments(int q, const double* u, const double* F, double phi, double* S);
/* g^eq (Eq. 42) and n^eq (Eq. 37) */
int ref_geq(double T, const double* u, double sigma, double varpi, double* geq);
int ref_neq(double T, const double* u, double sigma, double varpi, double* neq);
/* velocity closure (Eqs. 27-28): u from sum_i e_i f_i and G */
int ref_velocity(int q, const double* f, const double* G, double phi, double nu, double K,
                 double F_phi, double* u);
/* total force (Eq. 4) */
int ref_total_force(const double* u, const double* G, double phi, double nu, double K,
                    double F_phi, double* F);
/* threads the time loop uses (OpenMP over nodes) */
int ref_threads(void);
/* SplitMix64 output for state (seed ^ n) and the uniform noise drawn from it */
uint64_t ref_splitmix64(uint64_t state);
double ref_noise(uint64_t seed, uint64_t n, double amp);

/* ---- enthalpy-based D3Q7-MRT model, App. B, conduction only (enthalpy_oracle.c) */
typedef struct {
  int32_t nx, ny, nz;
  double varpi;                 /* csT^2 = varpi/3 (Eq. 40) */
  double porosity;              /* phi of Eq. B4 */
  double c_pl, c_ps;            /* specific heats of the liquid and the solid */
  double matrix_heat;           /* rho_m c_pm / (rho_l c_pl) of the porous matrix */
  double latent;                /* L_a */
  double T_solidus, T_liquidus; /* T_s <= T_l (Eq. B8) */
  double alpha_l, alpha_s;      /* effective diffusivities of each phase (Eq. B11, Sec. 4.3) */
  double zeta_e, zeta_nu;       /* rates of the non-conserved moments 4-6 (Eq. 38) */
  int32_t heat[6];              /* per face: 0 periodic, 1 adiabatic, 2 isothermal at T_wall */
  double T_wall[6];
  double T_init;                /* uniform initial temperature */
} ref_enthalpy_params;

typedef struct ref_enthalpy ref_enthalpy;
int ref_enthalpy_create(const ref_enthalpy_params* p, ref_enthalpy** out);
void ref_enthalpy_destroy(ref_enthalpy* h);
int64_t ref_enthalpy_time(const ref_enthalpy* h);
int ref_enthalpy_step(ref_enthalpy* h, int64_t nsteps);
/* T, En, f_l per node (any pointer may be NULL) */
int ref_enthalpy_fields(const ref_enthalpy* h, double* T, double* En, double* fl);
/* g in [7][z][y][x] */
int ref_enthalpy_get_state(const ref_enthalpy* h, double* g);
int ref_enthalpy_set_state(ref_enthalpy* h, const double* g);
/* T and f_l of an effective enthalpy (Eqs. B8, B9) */
int ref_enthalpy_phase(const ref_enthalpy* h, double En, double* T, double* fl);

#ifdef __cplusplus
}
#endif
#endif
