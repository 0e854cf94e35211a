// lbm_capi.hip -- host side of the C ABI declared in include/lbm.h: parameter
// validation and mapping (Eqs. 6, 7, 28, 32, 41, 51, 56), device memory layout,
// and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "lbm.h"
#include "kernels.hpp"

using namespace lbm;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static lbm_status fail(lbm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static lbm_status fail(lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(LBM_ERR_DEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                  \
  } while (0)

// ------------------------------------------------------------------ lattice
struct lbm_lattice {
  lbm_params p;
  lbm_derived d;
  hipStream_t stream = nullptr;
  void* buf = nullptr;
  bool owns_buf = false;
  size_t bytes = 0;
  int q = 19;
  int prec = LBM_FP64;
  int nodes = 0;
  int pstride = 0;
  int block = 256;
  int nblocks = 0;
  // carve-up of the device buffer
  void* state = nullptr;
  void* snap = nullptr;
  double* part = nullptr;
  double* part2 = nullptr;  // first-stage fold of part
  int nfold = 0;            // entries in part2
  double* res = nullptr;    // [0..7] residual, [8..13] wall flux, [16..17] totals
  int* dev_iso = nullptr;   // [6] isothermal flags
  double* dev_Tw = nullptr; // [6] wall temperatures
  double* host_res = nullptr; // pinned mirror of res (32 doubles)
  int parity = 0;
  int64_t t = 0;
  bool snapshot_valid = false;
  int64_t snapshot_at = -1;
  int64_t last_check = -1;
  KParams<double> kd;
  KParams<float> kf;
};

static constexpr double kCs2 = 1.0 / 3.0;

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ------------------------------------------------------------------ params
extern "C" void lbm_default_params(lbm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 8;
  p->lattice = 19;
  p->precision = LBM_FP64;
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
    p->face[k].flow = LBM_FLOW_WALL;
    p->face[k].heat = LBM_HEAT_ADIABATIC;
  }
  p->check_interval = 0;
}

static bool is_finite(double v) { return std::isfinite(v); }

// Validation and the parameter mapping of Sec. 4: Eq. 56 for a cavity (Ra, Pr, Ma),
// Eq. 51 read with 1/s_nu for a channel (Re, u_char), then Eqs. 32, 41, 7, 6, 28.
static lbm_status derive(const lbm_params* p, lbm_derived* d) {
  if (!p || !d) return fail(LBM_ERR_INVALID_ARG, "null parameter pointer");
  if (p->lattice != 19 && p->lattice != 15)
    return fail(LBM_ERR_INVALID_ARG, "lattice must be 19 or 15 (got %d)", p->lattice);
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32)
    return fail(LBM_ERR_UNSUPPORTED, "precision %d is not supported", p->precision);
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(LBM_ERR_INVALID_ARG, "box %dx%dx%d must have at least one node per axis", p->nx, p->ny, p->nz);
  const long long nodes = (long long)p->nx * p->ny * p->nz;
  if (nodes > (1ll << 30))
    return fail(LBM_ERR_INVALID_ARG, "box of %lld nodes exceeds the 2^30 node limit", nodes);
  if (!(p->porosity > 0.0 && p->porosity <= 1.0)) return fail(LBM_ERR_INVALID_ARG, "porosity must be in (0,1]");
  if (!(p->darcy > 0.0) || !is_finite(p->darcy)) return fail(LBM_ERR_INVALID_ARG, "darcy must be > 0");
  if (!(p->prandtl > 0.0) || !is_finite(p->prandtl)) return fail(LBM_ERR_INVALID_ARG, "prandtl must be > 0");
  if (!(p->delta_T > 0.0) || !is_finite(p->delta_T)) return fail(LBM_ERR_INVALID_ARG, "delta_T must be > 0");
  if (!(p->rayleigh >= 0.0) || !is_finite(p->rayleigh)) return fail(LBM_ERR_INVALID_ARG, "rayleigh must be >= 0");
  if (!(p->sigma > 0.0) || !(p->J > 0.0) || !(p->Gamma > 0.0))
    return fail(LBM_ERR_INVALID_ARG, "sigma, J and Gamma must be > 0");
  if (!(p->varpi > 0.0 && p->varpi < 1.0)) return fail(LBM_ERR_INVALID_ARG, "varpi must be in (0,1)");
  if (p->gravity_axis < 0 || p->gravity_axis > 2 || p->length_axis < 0 || p->length_axis > 2)
    return fail(LBM_ERR_INVALID_ARG, "gravity_axis and length_axis must be 0, 1 or 2");
  if (p->init_axis < -1 || p->init_axis > 2) return fail(LBM_ERR_INVALID_ARG, "init_axis must be -1, 0, 1 or 2");
  if (p->check_interval < 0) return fail(LBM_ERR_INVALID_ARG, "check_interval must be >= 0");
  for (int a = 0; a < 3; ++a) {
    const lbm_face& lo = p->face[2 * a];
    const lbm_face& hi = p->face[2 * a + 1];
    for (const lbm_face* f : {&lo, &hi}) {
      if (f->flow != LBM_FLOW_PERIODIC && f->flow != LBM_FLOW_WALL)
        return fail(LBM_ERR_UNSUPPORTED, "flow rule %d is not supported", f->flow);
      if (f->heat != LBM_HEAT_PERIODIC && f->heat != LBM_HEAT_ADIABATIC && f->heat != LBM_HEAT_ISOTHERMAL)
        return fail(LBM_ERR_UNSUPPORTED, "heat rule %d is not supported", f->heat);
      if ((f->flow == LBM_FLOW_PERIODIC) != (f->heat == LBM_HEAT_PERIODIC))
        return fail(LBM_ERR_INVALID_ARG, "a face must be periodic for both flow and heat, or for neither");
    }
    if ((lo.flow == LBM_FLOW_PERIODIC) != (hi.flow == LBM_FLOW_PERIODIC))
      return fail(LBM_ERR_INVALID_ARG, "opposite faces of axis %d must both be periodic or both not", a);
  }
  const int dims[3] = {p->nx, p->ny, p->nz};
  const double L = dims[p->length_axis];
  const double csT2 = p->varpi / 3.0;
  double s_nu;
  if (p->s_nu_set > 0.0) {
    s_nu = p->s_nu_set;
  } else if (p->reynolds > 0.0) {
    const double nu = p->u_char * L / p->reynolds;  // Re = L u_c / nu (Eq. 7)
    s_nu = 1.0 / (0.5 + p->J * nu / kCs2);           // Eq. 51 (inverse), Eq. 32
  } else {
    if (!(p->rayleigh > 0.0))
      return fail(LBM_ERR_INVALID_ARG, "Eq. 56 needs rayleigh > 0 unless s_nu_set is given");
    s_nu = 1.0 / (0.5 + p->mach * p->J * L * std::sqrt(3.0 * p->prandtl) / std::sqrt(p->rayleigh)); // Eq. 56
  }
  double zeta_a;
  if (p->zeta_alpha_set > 0.0) {
    zeta_a = p->zeta_alpha_set;
  } else {
    zeta_a = 1.0 / (0.5 + p->Gamma * kCs2 * (1.0 / s_nu - 0.5) / (p->J * p->sigma * csT2 * p->prandtl)); // Eq. 56
  }
  if (!(s_nu > 0.0 && s_nu < 2.0)) return fail(LBM_ERR_INVALID_ARG, "s_nu = %g is outside (0,2)", s_nu);
  if (!(zeta_a > 0.0 && zeta_a < 2.0)) return fail(LBM_ERR_INVALID_ARG, "zeta_alpha = %g is outside (0,2)", zeta_a);
  d->L = L;
  d->s_nu = s_nu;
  d->zeta_alpha = zeta_a;
  d->nu_e = kCs2 * (1.0 / s_nu - 0.5);                 // Eq. 32
  d->nu = d->nu_e / p->J;                              // J = nu_e / nu
  d->alpha_e = p->sigma * csT2 * (1.0 / zeta_a - 0.5); // Eq. 41
  d->alpha = d->alpha_e / p->Gamma;                    // Gamma = alpha_e / alpha
  d->K = p->darcy * L * L;                             // Da = K / L^2
  d->F_phi = p->forchheimer * 1.75 / std::sqrt(150.0 * p->porosity * p->porosity * p->porosity); // Eq. 6
  d->gbeta = p->rayleigh * d->nu * d->alpha / (L * L * L) / p->delta_T;  // Ra of Eq. 7
  d->l0 = 0.5 * (1.0 + p->porosity * 0.5 * d->nu / d->K);                // Eq. 28
  d->l1 = p->porosity * 0.5 * d->F_phi / std::sqrt(d->K);
  return LBM_OK;
}

// Rates of Eq. 22 (D3Q19) / Eq. 16 (D3Q15) and Eq. 38.
template <class C>
static void fill_kparams(const lbm_params* p, const lbm_derived* d, int nodes, int pstride, KParams<C>* k) {
  std::memset(k, 0, sizeof(*k));
  k->nx = p->nx;
  k->ny = p->ny;
  k->nz = p->nz;
  k->nxy = p->nx * p->ny;
  k->n = nodes;
  k->pstride = pstride;
  k->gaxis = p->gravity_axis;
  k->moving = 0;
  for (int a = 0; a < 3; ++a) k->per[a] = p->face[2 * a].flow == LBM_FLOW_PERIODIC;
  const double w7 = p->varpi / 6.0;
  for (int f = 0; f < 6; ++f) {
    for (int a = 0; a < 3; ++a) {
      const double u = p->face[f].flow == LBM_FLOW_WALL ? p->face[f].u_wall[a] : 0.0;
      k->u_wall[f][a] = (C)u;
      if (u != 0.0) k->moving = 1;
    }
    if (p->face[f].heat == LBM_HEAT_ISOTHERMAL) {
      // shifted anti-bounce-back: p_in = -p_out + 2 omega sigma (T_w - T_ref)
      k->heat_a[f] = (C)-1.0;
      k->heat_b[f] = (C)(2.0 * w7 * p->sigma * (p->face[f].T_wall - p->T_ref));
    } else {
      k->heat_a[f] = (C)1.0;
      k->heat_b[f] = (C)0.0;
    }
  }
  k->phi = (C)p->porosity;
  k->inv_phi = (C)(1.0 / p->porosity);
  k->c_darcy = (C)(p->porosity * d->nu / d->K);
  k->c_forch = (C)(p->porosity * d->F_phi / std::sqrt(d->K));
  k->l0 = (C)d->l0;
  k->l1 = (C)d->l1;
  k->gbeta = (C)d->gbeta;
  for (int a = 0; a < 3; ++a) k->accel[a] = (C)p->accel[a];
  k->sigma = (C)p->sigma;
  k->inv_sigma = (C)(1.0 / p->sigma);
  k->T_ref = (C)p->T_ref;
  k->varpi = (C)p->varpi;
  double s[19];
  if (p->lattice == 19) {
    const double r[19] = {p->s_rho, p->s_e,   p->s_eps, p->s_j,    p->s_q,   p->s_j,    p->s_q,
                          p->s_j,   p->s_q,   d->s_nu,  p->s_pi,   d->s_nu,  p->s_pi,   d->s_nu,
                          d->s_nu,  d->s_nu,  p->s_m,   p->s_m,    p->s_m};
    std::memcpy(s, r, sizeof r);
  } else {
    const double r[15] = {p->s_rho, p->s_e, p->s_eps, p->s_j,  p->s_q,  p->s_j,  p->s_q, p->s_j,
                          p->s_q,   d->s_nu, d->s_nu, d->s_nu, d->s_nu, d->s_nu, p->s_m};
    for (int i = 0; i < 19; ++i) s[i] = i < 15 ? r[i] : 0.0;
  }
  for (int i = 0; i < 19; ++i) {
    k->s[i] = (C)s[i];
    k->sh[i] = (C)(1.0 - 0.5 * s[i]);
  }
  const double z[7] = {p->zeta_T, d->zeta_alpha, d->zeta_alpha, d->zeta_alpha, p->zeta_e, p->zeta_nu, p->zeta_nu};
  for (int i = 0; i < 7; ++i) k->zeta[i] = (C)z[i];
  k->inv_dT = (C)(1.0 / p->delta_T);
}

// Device layout: [state | snapshot | partials | results | flags].
struct Layout {
  size_t state, snap, part, part2, res, iso, Tw, total;
  int pstride, nblocks, block, nfold;
};

static Layout layout(const lbm_params* p) {
  Layout L;
  const long long nodes = (long long)p->nx * p->ny * p->nz;
  const size_t s = p->precision == LBM_FP64 ? 8 : 4;
  L.block = 256;
  L.nblocks = (int)((nodes + L.block - 1) / L.block);
  // population planes start on 256-byte boundaries
  L.pstride = (int)align_up((size_t)nodes, 256 / s);
  size_t off = 0;
  L.state = off;
  off += align_up((size_t)(p->lattice + 7) * L.pstride * s, 256);
  L.snap = off;
  off += align_up((size_t)4 * nodes * s, 256);
  L.part = off;
  off += align_up((size_t)L.nblocks * kPartStride * sizeof(double), 256);
  L.nfold = (L.nblocks + L.block - 1) / L.block;
  L.part2 = off;
  off += align_up((size_t)L.nfold * kPartStride * sizeof(double), 256);
  L.res = off;
  off += 256;
  L.iso = off;
  off += 256;
  L.Tw = off;
  off += 256;
  L.total = off;
  return L;
}

extern "C" lbm_status lbm_required_bytes(const lbm_params* p, size_t* bytes) {
  if (!bytes) return fail(LBM_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = 0;
  lbm_derived d;
  lbm_status s = derive(p, &d);
  if (s != LBM_OK) return s;
  *bytes = layout(p).total;
  return LBM_OK;
}

// ------------------------------------------------------------------ dispatch
template <class F>
static void with_types(const lbm_lattice* h, F&& f) {
  if (h->q == 19) {
    if (h->prec == LBM_FP64) f(D3Q19{}, double{}, double{}, h->kd);
    else f(D3Q19{}, float{}, float{}, h->kf);
  } else {
    if (h->prec == LBM_FP64) f(D3Q15{}, double{}, double{}, h->kd);
    else f(D3Q15{}, float{}, float{}, h->kf);
  }
}

static lbm_status launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBM_ERR_DEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

extern "C" lbm_status lbm_create(const lbm_params* p, void* dev_buf, size_t bytes, void* stream,
                                 lbm_lattice** out) {
  if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  lbm_derived d;
  lbm_status s = derive(p, &d);
  if (s != LBM_OK) return s;
  const Layout L = layout(p);
  if (dev_buf) {
    if (bytes < L.total)
      return fail(LBM_ERR_OUT_OF_MEMORY, "buffer of %zu bytes is smaller than the %zu required", bytes, L.total);
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255) != 0)
      return fail(LBM_ERR_INVALID_ARG, "device buffer must be 256-byte aligned");
  }
  lbm_lattice* h = new (std::nothrow) lbm_lattice();
  if (!h) return fail(LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  h->p = *p;
  h->d = d;
  h->stream = (hipStream_t)stream;
  h->q = p->lattice;
  h->prec = p->precision;
  h->nodes = p->nx * p->ny * p->nz;
  h->pstride = L.pstride;
  h->block = L.block;
  h->nblocks = L.nblocks;
  if (dev_buf) {
    h->buf = dev_buf;
    h->bytes = bytes;
  } else {
    hipError_t e = hipMalloc(&h->buf, L.total);
    if (e != hipSuccess) {
      delete h;
      return fail(LBM_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed: %s", L.total, hipGetErrorString(e));
    }
    h->owns_buf = true;
    h->bytes = L.total;
  }
  hipError_t e = hipHostMalloc((void**)&h->host_res, 32 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    if (h->owns_buf) (void)hipFree(h->buf);
    delete h;
    return fail(LBM_ERR_OUT_OF_MEMORY, "hipHostMalloc failed: %s", hipGetErrorString(e));
  }
  std::memset(h->host_res, 0, 32 * sizeof(double));
  char* base = static_cast<char*>(h->buf);
  h->state = base + L.state;
  h->snap = base + L.snap;
  h->part = reinterpret_cast<double*>(base + L.part);
  h->part2 = reinterpret_cast<double*>(base + L.part2);
  h->nfold = L.nfold;
  h->res = reinterpret_cast<double*>(base + L.res);
  h->dev_iso = reinterpret_cast<int*>(base + L.iso);
  h->dev_Tw = reinterpret_cast<double*>(base + L.Tw);
  fill_kparams<double>(p, &d, h->nodes, h->pstride, &h->kd);
  fill_kparams<float>(p, &d, h->nodes, h->pstride, &h->kf);

  int iso[6];
  double Tw[6];
  for (int f = 0; f < 6; ++f) {
    iso[f] = p->face[f].heat == LBM_HEAT_ISOTHERMAL;
    Tw[f] = p->face[f].T_wall;
  }
  lbm_status st_ = LBM_OK;
  auto cleanup = [&]() {
    (void)hipHostFree(h->host_res);
    if (h->owns_buf) (void)hipFree(h->buf);
    delete h;
  };
  if (hipMemsetAsync(h->res, 0, 256, h->stream) != hipSuccess ||
      hipMemcpyAsync(h->dev_iso, iso, sizeof iso, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemcpyAsync(h->dev_Tw, Tw, sizeof Tw, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
    cleanup();
    return fail(LBM_ERR_DEVICE, "initial copies failed");
  }
  InitArgs ia{p->init_axis, p->init_T_lo, p->init_T_hi, p->seed, p->noise_amp};
  with_types(h, [&](auto lat, auto s_t, auto c_t, const auto& kp) {
    using Lat = decltype(lat);
    using S = decltype(s_t);
    using C = decltype(c_t);
    hipLaunchKernelGGL((k_init<Lat, S, C>), dim3(h->nblocks), dim3(h->block), 0, h->stream, kp, ia,
                       static_cast<S*>(h->state));
  });
  st_ = launch_check("init");
  if (st_ != LBM_OK) {
    cleanup();
    return st_;
  }
  // the copies above read host stack arrays: finish them before returning
  if (hipStreamSynchronize(h->stream) != hipSuccess) {
    cleanup();
    return fail(LBM_ERR_DEVICE, "stream synchronize failed during create");
  }
  *out = h;
  return LBM_OK;
}

extern "C" lbm_status lbm_destroy(lbm_lattice* h) {
  if (!h) return LBM_OK;
  lbm_status s = LBM_OK;
  if (hipStreamSynchronize(h->stream) != hipSuccess) s = fail(LBM_ERR_DEVICE, "stream synchronize failed");
  (void)hipHostFree(h->host_res);
  if (h->owns_buf) (void)hipFree(h->buf);
  delete h;
  return s;
}

extern "C" lbm_status lbm_set_stream(lbm_lattice* h, void* stream) {
  if (!h) return fail(LBM_ERR_INVALID_ARG, "lattice is NULL");
  h->stream = (hipStream_t)stream;
  return LBM_OK;
}

extern "C" lbm_status lbm_time(const lbm_lattice* h, int64_t* t) {
  if (!h || !t) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  *t = h->t;
  return LBM_OK;
}

extern "C" lbm_status lbm_derived_params(const lbm_lattice* h, lbm_derived* d) {
  if (!h || !d) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  *d = h->d;
  return LBM_OK;
}

// ------------------------------------------------------------------ step
template <class Lat, class S, class C>
static void launch_step(lbm_lattice* h, const KParams<C>& kp, int mode) {
  S* st_ = static_cast<S*>(h->state);
  C* sn = static_cast<C*>(h->snap);
  const dim3 g(h->nblocks), b(h->block);
  if (h->parity == 0) {
    if (mode == kModePlain) hipLaunchKernelGGL((k_step<Lat, S, C, false, kModePlain>), g, b, 0, h->stream, kp, st_, sn, h->part);
    else if (mode == kModeSnapshot) hipLaunchKernelGGL((k_step<Lat, S, C, false, kModeSnapshot>), g, b, 0, h->stream, kp, st_, sn, h->part);
    else hipLaunchKernelGGL((k_step<Lat, S, C, false, kModeCompare>), g, b, 0, h->stream, kp, st_, sn, h->part);
  } else {
    if (mode == kModePlain) hipLaunchKernelGGL((k_step<Lat, S, C, true, kModePlain>), g, b, 0, h->stream, kp, st_, sn, h->part);
    else if (mode == kModeSnapshot) hipLaunchKernelGGL((k_step<Lat, S, C, true, kModeSnapshot>), g, b, 0, h->stream, kp, st_, sn, h->part);
    else hipLaunchKernelGGL((k_step<Lat, S, C, true, kModeCompare>), g, b, 0, h->stream, kp, st_, sn, h->part);
  }
}

extern "C" lbm_status lbm_step(lbm_lattice* h, int64_t nsteps) {
  if (!h) return fail(LBM_ERR_INVALID_ARG, "lattice is NULL");
  if (nsteps < 0) return fail(LBM_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (h->host_res[7] != 0.0) return fail(LBM_ERR_UNSTABLE, "lattice was found unstable at an earlier check");
  const int64_t K = h->p.check_interval;
  for (int64_t s = 0; s < nsteps; ++s) {
    int mode = kModePlain;
    const int64_t t = h->t;
    if (K > 0) {
      if ((t + 1) % K == 0) mode = kModeSnapshot;
      else if (t > 0 && t % K == 0 && h->snapshot_valid && h->snapshot_at == t - 1) mode = kModeCompare;
    }
    with_types(h, [&](auto lat, auto s_t, auto c_t, const auto& kp) {
      launch_step<decltype(lat), decltype(s_t), decltype(c_t)>(h, kp, mode);
    });
    lbm_status ls = launch_check("step");
    if (ls != LBM_OK) return ls;
    if (mode == kModeSnapshot) {
      h->snapshot_valid = true;
      h->snapshot_at = t;
    }
    if (mode == kModeCompare) {
      hipLaunchKernelGGL(k_fold_partials, dim3(h->nfold), dim3(h->block), 0, h->stream, h->part, h->nblocks,
                         1u << 4, h->part2);
      hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, h->stream, h->part2, h->nfold, h->res);
      ls = launch_check("residual");
      if (ls != LBM_OK) return ls;
      HIP_TRY(hipMemcpyAsync(h->host_res, h->res, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      h->last_check = t;
      h->snapshot_valid = false;
    }
    h->parity ^= 1;
    h->t = t + 1;
  }
  return LBM_OK;
}

// ------------------------------------------------------------------ queries
extern "C" lbm_status lbm_fields(lbm_lattice* h, double* rho, double* ux, double* uy, double* uz, double* T) {
  if (!h) return fail(LBM_ERR_INVALID_ARG, "lattice is NULL");
  with_types(h, [&](auto lat, auto s_t, auto c_t, const auto& kp) {
    using Lat = decltype(lat);
    using S = decltype(s_t);
    using C = decltype(c_t);
    const S* st_ = static_cast<const S*>(h->state);
    if (h->parity)
      hipLaunchKernelGGL((k_fields<Lat, S, C, true>), dim3(h->nblocks), dim3(h->block), 0, h->stream, kp, st_, rho, ux, uy, uz, T);
    else
      hipLaunchKernelGGL((k_fields<Lat, S, C, false>), dim3(h->nblocks), dim3(h->block), 0, h->stream, kp, st_, rho, ux, uy, uz, T);
  });
  return launch_check("fields");
}

extern "C" lbm_status lbm_nusselt(lbm_lattice* h, double nu[6]) {
  if (!h || !nu) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  with_types(h, [&](auto lat, auto s_t, auto c_t, const auto& kp) {
    using Lat = decltype(lat);
    using S = decltype(s_t);
    using C = decltype(c_t);
    const S* st_ = static_cast<const S*>(h->state);
    if (h->parity)
      hipLaunchKernelGGL((k_wall_flux<Lat, S, C, true>), dim3(6), dim3(256), 0, h->stream, kp, st_, h->dev_iso, h->dev_Tw, h->res + 8);
    else
      hipLaunchKernelGGL((k_wall_flux<Lat, S, C, false>), dim3(6), dim3(256), 0, h->stream, kp, st_, h->dev_iso, h->dev_Tw, h->res + 8);
  });
  lbm_status ls = launch_check("wall flux");
  if (ls != LBM_OK) return ls;
  HIP_TRY(hipMemcpyAsync(h->host_res + 8, h->res + 8, 6 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int dims[3] = {h->p.nx, h->p.ny, h->p.nz};
  for (int f = 0; f < 6; ++f) {
    const int a = f / 2;
    const double cnt = (double)dims[(a + 1) % 3] * dims[(a + 2) % 3];
    nu[f] = h->p.face[f].heat == LBM_HEAT_ISOTHERMAL
                ? h->host_res[8 + f] / cnt * h->d.L / (h->d.alpha_e * h->p.delta_T)
                : 0.0;
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_residual(lbm_lattice* h, double* r, int64_t* at_step) {
  if (!h || !r || !at_step) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (h->last_check < 0) {
    *r = -1.0;
    *at_step = -1;
  } else {
    *r = h->host_res[0];
    *at_step = h->last_check;
  }
  if (h->host_res[7] != 0.0) return fail(LBM_ERR_UNSTABLE, "a residual check found a non-finite value or |u| > 0.5");
  return LBM_OK;
}

extern "C" lbm_status lbm_totals(lbm_lattice* h, double* mass, double* heat) {
  if (!h) return fail(LBM_ERR_INVALID_ARG, "lattice is NULL");
  with_types(h, [&](auto lat, auto s_t, auto c_t, const auto& kp) {
    using Lat = decltype(lat);
    using S = decltype(s_t);
    using C = decltype(c_t);
    const S* st_ = static_cast<const S*>(h->state);
    if (h->parity)
      hipLaunchKernelGGL((k_totals<Lat, S, C, true>), dim3(h->nblocks), dim3(h->block), 0, h->stream, kp, st_, h->part);
    else
      hipLaunchKernelGGL((k_totals<Lat, S, C, false>), dim3(h->nblocks), dim3(h->block), 0, h->stream, kp, st_, h->part);
  });
  lbm_status ls = launch_check("totals");
  if (ls != LBM_OK) return ls;
  hipLaunchKernelGGL(k_fold_partials, dim3(h->nfold), dim3(h->block), 0, h->stream, h->part, h->nblocks, 0u,
                     h->part2);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, h->stream, h->part2, h->nfold, h->res + 16);
  ls = launch_check("totals final");
  if (ls != LBM_OK) return ls;
  HIP_TRY(hipMemcpyAsync(h->host_res + 16, h->res + 16, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  // a compare step that follows reuses the partials buffer, so the snapshot stays valid
  if (mass) *mass = (double)h->nodes + h->host_res[16];
  if (heat) *heat = (double)h->nodes * h->p.sigma * h->p.T_ref + h->host_res[17];
  return LBM_OK;
}

extern "C" lbm_status lbm_get_state(lbm_lattice* h, double* f, double* g) {
  if (!h) return fail(LBM_ERR_INVALID_ARG, "lattice is NULL");
  with_types(h, [&](auto lat, auto s_t, auto c_t, const auto& kp) {
    using Lat = decltype(lat);
    using S = decltype(s_t);
    using C = decltype(c_t);
    const S* st_ = static_cast<const S*>(h->state);
    if (h->parity)
      hipLaunchKernelGGL((k_get_state<Lat, S, C, true>), dim3(h->nblocks), dim3(h->block), 0, h->stream, kp, st_, f, g);
    else
      hipLaunchKernelGGL((k_get_state<Lat, S, C, false>), dim3(h->nblocks), dim3(h->block), 0, h->stream, kp, st_, f, g);
  });
  return launch_check("get_state");
}

extern "C" lbm_status lbm_set_state(lbm_lattice* h, const double* f, const double* g) {
  if (!h || !f || !g) return fail(LBM_ERR_INVALID_ARG, "lbm_set_state needs both f and g");
  with_types(h, [&](auto lat, auto s_t, auto c_t, const auto& kp) {
    using Lat = decltype(lat);
    using S = decltype(s_t);
    using C = decltype(c_t);
    hipLaunchKernelGGL((k_set_state<Lat, S, C>), dim3(h->nblocks), dim3(h->block), 0, h->stream, kp,
                       static_cast<S*>(h->state), f, g);
  });
  lbm_status ls = launch_check("set_state");
  if (ls != LBM_OK) return ls;
  h->parity = 0;
  h->snapshot_valid = false;
  return LBM_OK;
}

extern "C" const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_INVALID_ARG: return "invalid argument";
    case LBM_ERR_OUT_OF_MEMORY: return "out of memory";
    case LBM_ERR_DEVICE: return "device error";
    case LBM_ERR_UNSTABLE: return "unstable";
    case LBM_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

extern "C" const char* lbm_last_error(void) { return g_last_error.c_str(); }
