// C ABI of the library: contexts, columns (validation, device layout and the
// n-independent setup of Sect. 2.1.1), residual and Jacobian-vector product.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "nlte_internal.h"
#include "voigt.h"

using namespace nlte;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

nlte_status set_err(nlte_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

extern "C" const char* nlte_last_error(void) { return g_err.c_str(); }

#define HIP_TRY(x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return set_err(NLTE_E_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_));       \
  } while (0)

// ---------------------------------------------------------------------------
// context and column objects
// ---------------------------------------------------------------------------
struct nlte_column {
  nlte_ctx* ctx = nullptr;
  int device = 0;             // ctx->device, kept so that destruction never reads ctx
  ColDev h{};                 // device pointers, host copy
  ColDev* d = nullptr;        // device copy (one-element batch)
  void* arena = nullptr;
  size_t arena_bytes = 0;
  BatchWork bw;               // single-column work lists (col index 0)
  int restart_cap = 0;
  std::vector<double> Blu;    // host copy of line B_lu (profile-averaged J)
  bool pooled = false;        // arena (with d at its end) lent by a server's pool: not freed here
};

namespace nlte {
const ColDev& column_dev(const nlte_column* c) { return c->h; }
ColDev* column_dev_ptr(const nlte_column* c) { return c->d; }
int column_restart_cap(const nlte_column* c) { return c->restart_cap; }
nlte_ctx* column_ctx(const nlte_column* c) { return c->ctx; }
size_t column_bytes(const nlte_column* c) { return c->arena_bytes; }
}  // namespace nlte

// ---------------------------------------------------------------------------
// device-resident scratch of the allocation-free residual entry point
// ---------------------------------------------------------------------------
// One fixed array per device, held until the process ends.  In host code its
// name is only a host-side stand-in: kernels get the device address that
// hipGetSymbolAddress returns for each device (scratch_base).
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];

struct ScratchSlot {
  std::once_flag once;
  char* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[kMaxDevices];

// Looks the array's address up once per device (that device current).
void scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  ScratchSlot& S = g_scratch[dev];
  std::call_once(S.once, [&S] {
    void* p = nullptr;
    S.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (S.err == hipSuccess) S.ptr = static_cast<char*>(p);
  });
}

char* scratch_base(int dev, hipError_t* err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  scratch_init(dev);
  *err = g_scratch[dev].err;
  return g_scratch[dev].ptr;
}
}  // namespace

extern "C" nlte_status nlte_ctx_create(int hip_device, nlte_ctx** out) {
  if (!out) return set_err(NLTE_E_INVALID, "out is NULL");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev)
    return set_err(NLTE_E_INVALID, "device %d out of range (%d devices)", hip_device, ndev);
  HIP_TRY(hipSetDevice(hip_device));
  scratch_init(hip_device);  // errors are reported by the entry point that needs it
  nlte_ctx* c = new nlte_ctx();
  c->device = hip_device;
  c->prof_on = 0;
  memset(&c->prof, 0, sizeof c->prof);
  *out = c;
  return NLTE_OK;
}

extern "C" void nlte_ctx_destroy(nlte_ctx* ctx) { delete ctx; }

extern "C" nlte_status nlte_profile_enable(nlte_ctx* ctx, int on) {
  if (!ctx) return set_err(NLTE_E_INVALID, "NULL ctx");
  ctx->prof_on = on != 0;
  memset(&ctx->prof, 0, sizeof ctx->prof);
  return NLTE_OK;
}

extern "C" nlte_status nlte_profile_read(const nlte_ctx* ctx, nlte_profile* out) {
  if (!ctx || !out) return set_err(NLTE_E_INVALID, "NULL argument");
  *out = ctx->prof;
  return NLTE_OK;
}

extern "C" void nlte_solve_opts_default(nlte_solve_opts* o) {
  if (!o) return;
  o->ftol = 1e-8;
  o->rtol = 1e-3;
  o->maxiter = 50;
  o->max_krylov = 200;
  o->max_krylov_total = 0;
  o->fp64_fallback = 0;
  o->restart = 30;
  o->max_halvings = 8;
  o->init = 1;
  o->eps_scale = 1.0;
  o->krylov_method = NLTE_KRYLOV_GMRES;
  o->jv_method = NLTE_JV_FD;
  o->krylov_x0 = 0;
  o->launch = 0;
}

// ---------------------------------------------------------------------------
// arena layout
// ---------------------------------------------------------------------------
namespace {
struct Layout {
  char* base;
  size_t off = 0;
  explicit Layout(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// raw inputs that only the setup kernels read
struct SetupIn {
  const double *E, *g, *A_ul, *a_damp, *bf_nu, *bf_alpha, *C_up;
  const double *w_nu;  // caller frequency weights [nnu] or NULL (trapezoid per window)
  const int *stage, *bf_ptr;
  double mass_amu, vturb;
  double mu[kMaxMu];   // angle cosines (Doppler shifts of the rays)
};

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(p[i])) return false;
  return true;
}
}  // namespace

// ---------------------------------------------------------------------------
// setup kernels (n-independent tables, Sect. 2.1.1)
// ---------------------------------------------------------------------------
// Per depth: LTE populations (Saha-Boltzmann), n*_l/n*_c of each edge,
// downward collision rates by detailed balance, depth steps.
__global__ void k_setup_depth(ColDev C, SetupIn in) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= C.nz) return;
  const int L = C.L;
  const double T = C.T[k];
  const double saha = log(2.0 * pow(2.0 * kPi * kMe * kK * T / (kH * kH), 1.5) / C.ne[k]);
  double lw[kMaxLev];
  double mx = -1e300;
  for (int i = 0; i < L; ++i) {
    lw[i] = log(in.g[i]) - in.E[i] / (kK * T) + in.stage[i] * saha;
    mx = fmax(mx, lw[i]);
  }
  double s = 0.0;
  for (int i = 0; i < L; ++i) {
    lw[i] = exp(lw[i] - mx);
    s += lw[i];
  }
  double* ns = (double*)C.nstar + k * L;
  for (int i = 0; i < L; ++i) ns[i] = C.ntot[k] * lw[i] / s;
  for (int e = 0; e < C.nbf; ++e) {
    const TrDev T_ = C.tr[C.nline + e];
    ((double*)C.rho_bf)[k * C.nbf + e] = ns[T_.lo] / ns[T_.up];
  }
  for (int t = 0; t < C.ntr; ++t) {
    const TrDev T_ = C.tr[t];
    const double cu = in.C_up[k * C.ntr + t];
    ((double*)C.C_lu)[k * C.ntr + t] = cu;
    ((double*)C.C_ul)[k * C.ntr + t] = cu * ns[T_.lo] / ns[T_.up];
  }
  if (k + 1 < C.nz) ((double*)C.dz)[k] = fabs(C.z[k + 1] - C.z[k]);
}

// Per (k, f): Planck function, exp(-h nu/kT), and 2 h nu^3 / c^2.
__global__ void k_setup_freq(ColDev C) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)C.nz * C.nnu) return;
  const int k = (int)(i / C.nnu), f = (int)(i % C.nnu);
  const double nu = C.nu[f];
  const double x = kH * nu / (kK * C.T[k]);
  const double gam = 2.0 * kH * nu * nu * nu / (kC * kC);
  ((double*)C.Bnu)[i] = gam / expm1(x);
  if (C.nbf) ((double*)C.Ebf)[i] = exp(-x);
  if (k == 0) ((double*)C.gam)[f] = gam;
  C.Jdag[i] = gam / expm1(x);
}

// Per (t, window point): rate weight 4 pi w/(h nu) with trapezoid weights
// over the transition's own window (or the caller's weights); edges:
// cross-section interpolated linearly onto the union grid (their V table).
__global__ void k_setup_window(ColDev C, SetupIn in, const int* __restrict__ wbase, int wtotal) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= wtotal) return;
  int t = 0;
  while (t + 1 < C.ntr && wbase[t + 1] <= i) ++t;
  const TrDev T = C.tr[t];
  const int fl = i - wbase[t];
  const int f = T.wlo + fl;
  const int fm = max(f - 1, T.wlo), fp = min(f + 1, T.whi - 1);
  const double w = in.w_nu ? in.w_nu[f] : 0.5 * (C.nu[fp] - C.nu[fm]);
  ((double*)C.cw)[T.cwoff + fl] = 4.0 * kPi * w / (kH * C.nu[f]);
  if (t >= C.nline) {
    const int e = t - C.nline;
    const int p0 = in.bf_ptr[e], p1 = in.bf_ptr[e + 1];
    const double nu = C.nu[f];
    double a;
    if (nu <= in.bf_nu[p0]) a = in.bf_alpha[p0];
    else if (nu >= in.bf_nu[p1 - 1]) a = in.bf_alpha[p1 - 1];
    else {
      int lo = p0, hi = p1 - 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (in.bf_nu[mid] <= nu) lo = mid; else hi = mid;
      }
      const double s = (nu - in.bf_nu[lo]) / (in.bf_nu[hi] - in.bf_nu[lo]);
      a = in.bf_alpha[lo] + s * (in.bf_alpha[hi] - in.bf_alpha[lo]);
    }
    ((double*)C.V)[T.voff + fl] = a;
  }
}

// Per (line, k, window point): raw Voigt profile value H(a, v).
__global__ void k_setup_voigt(ColDev C, SetupIn in, const int* __restrict__ lbase, int ltotal) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)ltotal * C.nz) return;
  const int k = (int)(i / ltotal);
  const int j = (int)(i % ltotal);
  int t = 0;
  while (t + 1 < C.nline && lbase[t + 1] <= j) ++t;
  const TrDev T = C.tr[t];
  const int fl = j - lbase[t];
  const int wl = T.whi - T.wlo;
  const double nu0 = (in.E[T.up] - in.E[T.lo]) / kH;
  const double dnuD = nu0 / kC * sqrt(2.0 * kK * C.T[k] / (in.mass_amu * kAmu) + in.vturb * in.vturb);
  const double v = (C.nu[T.wlo + fl] - nu0) / dnuD;
  ((double*)C.V)[T.voff + (size_t)k * wl + fl] = voigt_H(in.a_damp[t], v);
}

// Per (transition, k): profile normalisation on the window (lines),
// V = (h nu / 4 pi) B_lu phi, and the n-independent part of R_ul:
//   lines: sum_f cw V 2hnu^3/c^2;  edges: sum_f cw alpha exp(-h nu/kT) 2hnu^3/c^2.
__global__ void k_setup_norm(ColDev C, SetupIn in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C.ntr * C.nz) return;
  const int t = i / C.nz, k = i % C.nz;
  const TrDev T = C.tr[t];
  const int wl = T.whi - T.wlo;
  double rsp = 0.0;
  if (t < C.nline) {
    double* phi = (double*)C.V + T.voff + (size_t)k * wl;
    double s = 0.0;
    for (int fl = 0; fl < wl; ++fl) {
      const int f = T.wlo + fl;
      const int fm = max(f - 1, T.wlo), fp = min(f + 1, T.whi - 1);
      s += (in.w_nu ? in.w_nu[f] : 0.5 * (C.nu[fp] - C.nu[fm])) * phi[fl];
    }
    for (int fl = 0; fl < wl; ++fl) {
      const int f = T.wlo + fl;
      const double V = kH * C.nu[f] / (4.0 * kPi) * T.Blu * (phi[fl] / s);
      phi[fl] = V;
      rsp += C.cw[T.cwoff + fl] * V * C.gam[f];
    }
  } else {
    for (int fl = 0; fl < wl; ++fl) {
      const int f = T.wlo + fl;
      rsp += C.cw[T.cwoff + fl] * C.V[T.voff + fl] * C.Ebf[(size_t)k * C.nnu + f] * C.gam[f];
    }
  }
  ((double*)C.Rsp)[k * C.ntr + t] = rsp;
}

// Velocity fields (Sect. 3.5).  Per (ray, k, line window point): raw Voigt
// value of the profile the ray sees, centred on nu0 (1 + s mu v_k / c),
// s = +1 for the outgoing rays 0..nmu-1 and -1 for the ingoing ones.
__global__ void k_setup_voigt_vel(ColDev C, SetupIn in, const int* __restrict__ lbase, int ltotal) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)ltotal * C.nz * C.nray) return;
  const int j = (int)(i % ltotal);
  const size_t rest = i / ltotal;
  const int k = (int)(rest % C.nz), r = (int)(rest / C.nz);
  int t = 0;
  while (t + 1 < C.nline && lbase[t + 1] <= j) ++t;
  const TrDev T = C.tr[t];
  const int fl = j - lbase[t];
  const int wl = T.whi - T.wlo;
  const double nu0 = (in.E[T.up] - in.E[T.lo]) / kH;
  const double dnuD = nu0 / kC * sqrt(2.0 * kK * C.T[k] / (in.mass_amu * kAmu) + in.vturb * in.vturb);
  const double s = r < C.nmu ? 1.0 : -1.0;
  const double proj = s * in.mu[r < C.nmu ? r : r - C.nmu] * C.vlos[k];
  const double v = (C.nu[T.wlo + fl] - nu0 * (1.0 + proj / kC)) / dnuD;
  ((double*)C.VR)[(size_t)C.nray * T.voff + ((size_t)r * C.nz + k) * wl + fl] = voigt_H(in.a_damp[t], v);
}

// Per (line, ray, k): normalisation of the ray's profile on the window and
// V = (h nu / 4 pi) B_lu phi_ray.
__global__ void k_setup_norm_vel(ColDev C, SetupIn in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C.nline * C.nray * C.nz) return;
  const int t = i / (C.nray * C.nz), rk = i % (C.nray * C.nz);
  const TrDev T = C.tr[t];
  const int wl = T.whi - T.wlo;
  double* phi = (double*)C.VR + (size_t)C.nray * T.voff + (size_t)rk * wl;
  double s = 0.0;
  for (int fl = 0; fl < wl; ++fl) {
    const int f = T.wlo + fl;
    const int fm = max(f - 1, T.wlo), fp = min(f + 1, T.whi - 1);
    s += (in.w_nu ? in.w_nu[f] : 0.5 * (C.nu[fp] - C.nu[fm])) * phi[fl];
  }
  for (int fl = 0; fl < wl; ++fl)
    phi[fl] = kH * C.nu[T.wlo + fl] / (4.0 * kPi) * T.Blu * (phi[fl] / s);
}

// Per (line, k): the n-independent part of R_ul with the angle integral
// inside, sum_f cw (2 h nu^3/c^2) sum_rays (w_m/2) V_ray (replaces the
// static value written by k_setup_norm).
__global__ void k_setup_rsp_vel(ColDev C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C.nline * C.nz) return;
  const int t = i / C.nz, k = i % C.nz;
  const TrDev T = C.tr[t];
  const int wl = T.whi - T.wlo;
  const double* V = C.VR + (size_t)C.nray * T.voff + (size_t)k * wl;
  double rsp = 0.0;
  for (int fl = 0; fl < wl; ++fl) {
    double vb = 0.0;
    for (int r = 0; r < C.nray; ++r) vb += C.wm2[r < C.nmu ? r : r - C.nmu] * V[(size_t)r * C.nz * wl + fl];
    rsp += C.cw[T.cwoff + fl] * vb * C.gam[T.wlo + fl];
  }
  ((double*)C.Rsp)[k * C.ntr + t] = rsp;
}

// Depth-contiguous copies of the per-ray V tables (velocity fields):
// element (ray, k, q) of a line's [nray][nz][wl] block goes to (ray, q, k).
__global__ void k_setup_transpose_vel(ColDev C, size_t total) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int t = 0;
  while (t + 1 < C.nline && (size_t)C.nray * C.tr[t + 1].voff <= i) ++t;
  const TrDev T = C.tr[t];
  const size_t wl = T.whi - T.wlo, blk = (size_t)C.nz * wl;
  const size_t loc = i - (size_t)C.nray * T.voff;
  const size_t r = loc / blk, rem = loc % blk;
  const size_t k = rem / wl, q = rem % wl;
  ((double*)C.VRT)[(size_t)C.nray * T.voff + r * blk + q * C.nz + k] = C.VR[i];
}

// Depth-contiguous copies for the kernels that run one lane per depth.
__global__ void k_setup_transpose(ColDev C, int nline_tab_total) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t kf = (size_t)C.nz * C.nnu;
  if (C.nbf && i < kf) {
    const int k = (int)(i / C.nnu), f = (int)(i % C.nnu);
    ((double*)C.EbfT)[(size_t)f * C.zp + k] = C.Ebf[i];
  }
  if (i < (size_t)nline_tab_total) {
    // find the line owning element i of the packed [nz][wl] tables
    int t = 0;
    while (t + 1 < C.nline && (size_t)C.tr[t + 1].voff <= i) ++t;
    const TrDev T = C.tr[t];
    const int wl = T.whi - T.wlo;
    const size_t loc = i - T.voff;
    const int k = (int)(loc / wl), q = (int)(loc % wl);
    ((double*)C.VT)[T.voff + (size_t)q * C.nz + k] = C.V[i];
  }
}

// FP32 copies of the tables the FP32-form opacity kernel reads.
__global__ void k_setup_f32(ColDev C, size_t nv, size_t nvt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t kf = (size_t)C.nz * C.nnu;
  if (i < nv) ((float*)C.Vf)[i] = (float)C.V[i];
  if (i < nvt) ((float*)C.VTf)[i] = (float)C.VT[i];
  if (i < kf) {
    const size_t k = i / C.nnu, ip = k * C.fp + (i - k * C.nnu);  // padded rows
    ((float*)C.Bnuf)[ip] = (float)C.Bnu[i];
    if (C.bg_eta) ((float*)C.ECf)[ip] = (float)C.EC[i];
    if (C.nbf) {
      ((float*)C.Ebff)[ip] = (float)C.Ebf[i];
      const size_t f = i / C.nz, iz = f * C.zp + (i - f * C.nz);  // padded [nnu][zp]
      ((float*)C.EbfTf)[iz] = (float)C.EbfT[iz];
    }
  }
}

// J [nnu][nz] -> [nz][nnu]
__global__ void k_transpose_J(const double* __restrict__ JT, double* __restrict__ out, int nz, int nnu,
                              int zp) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)nz * nnu) return;
  const int k = (int)(i / nnu), f = (int)(i % nnu);
  out[i] = JT[(size_t)f * zp + k];
}

namespace nlte {
void transpose_J(const ColDev& C, double* out, hipStream_t s) {
  const size_t n = (size_t)C.nz * C.nnu;
  k_transpose_J<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(C.JT, out, C.nz, C.nnu, C.zp);
}
}  // namespace nlte

// ---------------------------------------------------------------------------
// column creation
// ---------------------------------------------------------------------------
static nlte_status validate(const nlte_atmos_desc* A, const nlte_atom_desc* M,
                            const nlte_grid_desc* G, const double* C_up) {
  if (!A || !M || !G || !C_up) return set_err(NLTE_E_INVALID, "NULL descriptor");
  const int nz = A->nz, L = M->nlev, nnu = G->nnu, nmu = G->nmu;
  if (nz < 3) return set_err(NLTE_E_INVALID, "nz = %d < 3", nz);
  if (L < 2 || L > kMaxLev) return set_err(NLTE_E_INVALID, "nlev = %d outside 2..%d", L, kMaxLev);
  if (nmu < 1 || nmu > kMaxMu) return set_err(NLTE_E_INVALID, "nmu = %d outside 1..%d", nmu, kMaxMu);
  if (nnu < 2) return set_err(NLTE_E_INVALID, "nnu = %d < 2", nnu);
  if (M->nline < 0 || M->nbf < 0 || M->nline + M->nbf < 1)
    return set_err(NLTE_E_INVALID, "need at least one transition");
  if (!A->z || !A->T || !A->ne || !A->ntot || !A->chi_c || !M->E || !M->g || !M->stage ||
      !G->nu || !G->win_lo || !G->win_hi || !G->mu || !G->w_mu)
    return set_err(NLTE_E_INVALID, "NULL array in descriptor");
  const double* zs[] = {A->z, A->T, A->ne, A->ntot, A->chi_c};
  for (auto p : zs)
    if (!finite_all(p, nz)) return set_err(NLTE_E_NONFINITE, "non-finite atmosphere value");
  if (A->chi_sca && !finite_all(A->chi_sca, nz)) return set_err(NLTE_E_NONFINITE, "non-finite chi_sca");
  if (A->vlos) {
    if (!finite_all(A->vlos, nz)) return set_err(NLTE_E_NONFINITE, "non-finite vlos");
    for (int k = 0; k < nz; ++k)
      if (!(fabs(A->vlos[k]) < 0.1 * kC)) return set_err(NLTE_E_INVALID, "|vlos[%d]| >= c/10", k);
  }
  if (A->eta_c) {
    if (!finite_all(A->eta_c, (size_t)nz * nnu)) return set_err(NLTE_E_NONFINITE, "non-finite eta_c");
    for (size_t i = 0; i < (size_t)nz * nnu; ++i)
      if (A->eta_c[i] < 0) return set_err(NLTE_E_INVALID, "negative eta_c");
  }
  if (G->w_nu) {
    if (!finite_all(G->w_nu, nnu)) return set_err(NLTE_E_NONFINITE, "non-finite w_nu");
    for (int f = 0; f < nnu; ++f)
      if (!(G->w_nu[f] > 0)) return set_err(NLTE_E_INVALID, "w_nu[%d] <= 0", f);
  }
  for (int k = 0; k < nz; ++k) {
    if (A->ntot[k] <= 0) return set_err(NLTE_E_INVALID, "ntot[%d] <= 0", k);
    if (A->T[k] <= 0) return set_err(NLTE_E_INVALID, "T[%d] <= 0", k);
    if (A->ne[k] <= 0) return set_err(NLTE_E_INVALID, "ne[%d] <= 0", k);
    if (A->chi_c[k] < 0 || (A->chi_sca && A->chi_sca[k] < 0))
      return set_err(NLTE_E_INVALID, "negative background opacity at %d", k);
    if (k + 1 < nz && !(A->z[k + 1] > A->z[k])) return set_err(NLTE_E_INVALID, "z not increasing at %d", k);
  }
  if (!finite_all(G->nu, nnu)) return set_err(NLTE_E_NONFINITE, "non-finite nu");
  for (int f = 0; f + 1 < nnu; ++f)
    if (!(G->nu[f + 1] > G->nu[f]) || G->nu[f] <= 0) return set_err(NLTE_E_INVALID, "nu not increasing at %d", f);
  double ws = 0;
  for (int m = 0; m < nmu; ++m) {
    if (!(G->mu[m] > 0 && G->mu[m] < 1)) return set_err(NLTE_E_INVALID, "mu[%d] outside (0,1)", m);
    if (!(G->w_mu[m] > 0)) return set_err(NLTE_E_INVALID, "w_mu[%d] <= 0", m);
    ws += G->w_mu[m];
  }
  if (fabs(ws - 1.0) > 1e-10) return set_err(NLTE_E_INVALID, "angle weights sum to %g, not 1", ws);
  if (!finite_all(M->E, L) || !finite_all(M->g, L)) return set_err(NLTE_E_NONFINITE, "non-finite level data");
  int ncont = 0;
  for (int i = 0; i < L; ++i) {
    if (M->g[i] <= 0) return set_err(NLTE_E_INVALID, "g[%d] <= 0", i);
    if (M->stage[i] != 0 && M->stage[i] != 1) return set_err(NLTE_E_INVALID, "stage[%d] not 0/1", i);
    ncont += M->stage[i];
  }
  const int ntr = M->nline + M->nbf;
  for (int t = 0; t < M->nline; ++t) {
    const int lo = M->line_lo[t], up = M->line_up[t];
    if (lo < 0 || up >= L || lo >= up || M->stage[lo] || M->stage[up])
      return set_err(NLTE_E_INVALID, "line %d levels (%d,%d) invalid", t, lo, up);
    if (!(M->E[up] > M->E[lo])) return set_err(NLTE_E_INVALID, "line %d has E_up <= E_lo", t);
    if (!(M->A_ul[t] > 0) || !isfinite(M->A_ul[t])) return set_err(NLTE_E_INVALID, "A_ul[%d] invalid", t);
    if (!(M->a_damp[t] >= 0 && M->a_damp[t] <= 0.1)) return set_err(NLTE_E_INVALID, "a_damp[%d] outside [0, 0.1]", t);
  }
  if (M->nline && !(M->mass_amu > 0)) return set_err(NLTE_E_INVALID, "mass_amu <= 0");
  if (M->nbf) {
    if (ncont != 1 || M->stage[L - 1] != 1)
      return set_err(NLTE_E_INVALID, "edges need exactly one continuum level, the last");
    for (int e = 0; e < M->nbf; ++e) {
      const int lo = M->bf_lo[e];
      if (lo < 0 || lo >= L - 1) return set_err(NLTE_E_INVALID, "edge %d lower level invalid", e);
      const int p0 = M->bf_ptr[e], p1 = M->bf_ptr[e + 1];
      if (p1 - p0 < 1 || p0 < 0) return set_err(NLTE_E_INVALID, "edge %d tabulation empty", e);
      for (int p = p0; p < p1; ++p) {
        if (!isfinite(M->bf_nu[p]) || !isfinite(M->bf_alpha[p]) || M->bf_alpha[p] < 0)
          return set_err(NLTE_E_INVALID, "edge %d cross-section invalid", e);
        if (p > p0 && !(M->bf_nu[p] > M->bf_nu[p - 1])) return set_err(NLTE_E_INVALID, "edge %d nu not increasing", e);
      }
    }
  }
  for (int t = 0; t < ntr; ++t) {
    if (G->win_lo[t] < 0 || G->win_hi[t] > nnu || G->win_hi[t] - G->win_lo[t] < 2)
      return set_err(NLTE_E_INVALID, "window of transition %d invalid", t);
  }
  if (!finite_all(C_up, (size_t)nz * ntr)) return set_err(NLTE_E_NONFINITE, "non-finite collision rate");
  for (size_t i = 0; i < (size_t)nz * ntr; ++i)
    if (C_up[i] < 0) return set_err(NLTE_E_INVALID, "negative collision rate");
  return NLTE_OK;
}

struct WorkPtrs {
  Tile* tiles;
  int4* rate;
  int2* pb;
};

static void layout_column(Layout& Lo, ColDev& C, SetupIn& in, int nwin_total, int nline_tab,
                          int nbf_tot, int nentries, int nentries_e, int m_cap, TrDev** tr_out, int** wbase,
                          int** lbase, WorkPtrs* wp, const int* wsz, int** stage, int** bf_ptr,
                          double** raw) {
  const int nz = C.nz, L = C.L, ntr = C.ntr, nnu = C.nnu, N = C.N;
  const size_t kf = (size_t)nz * nnu, kfp = (size_t)nz * C.fp, kfz = (size_t)nnu * C.zp;
  C.st = Lo.take<ColState>(1);
  C.z = Lo.take<double>(nz);
  C.dz = Lo.take<double>(nz);
  C.T = Lo.take<double>(nz);
  C.ne = Lo.take<double>(nz);
  C.ntot = Lo.take<double>(nz);
  C.chi_c = Lo.take<double>(nz);
  C.chi_sca = Lo.take<double>(nz);
  C.nu = Lo.take<double>(nnu);
  C.gam = Lo.take<double>(nnu);
  C.Bnu = Lo.take<double>(kf);
  C.EC = C.bg_eta ? Lo.take<double>(kf) : C.Bnu;
  C.Ebf = C.nbf ? Lo.take<double>(kf) : nullptr;
  C.EbfT = C.nbf ? Lo.take<double>(kfz) : nullptr;
  *tr_out = Lo.take<TrDev>(ntr);
  C.tr = *tr_out;
  C.V = Lo.take<double>((size_t)nline_tab * nz + (nwin_total - nline_tab));
  C.VT = Lo.take<double>((size_t)nline_tab * nz + 1);
  C.cw = Lo.take<double>(nwin_total);
  C.rho_bf = Lo.take<double>((size_t)nz * std::max(C.nbf, 1));
  C.Rsp = Lo.take<double>((size_t)nz * ntr);
  C.C_lu = Lo.take<double>((size_t)nz * ntr);
  C.C_ul = Lo.take<double>((size_t)nz * ntr);
  C.nstar = Lo.take<double>((size_t)nz * L);
  C.ch_lptr = Lo.take<int>(C.nchunk + 1);
  C.ch_line = Lo.take<int>(nentries);
  C.ch_eptr = Lo.take<int>(C.nchunk + 1);
  C.ch_edge = Lo.take<int>(nentries_e);
  if (C.prec == NLTE_FP32_FORM) {
    C.Vf = Lo.take<float>((size_t)nline_tab * nz + (nwin_total - nline_tab));
    C.Bnuf = Lo.take<float>(kfp);
    C.ECf = C.bg_eta ? Lo.take<float>(kfp) : C.Bnuf;
    C.Ebff = C.nbf ? Lo.take<float>(kfp) : nullptr;
    C.VTf = Lo.take<float>((size_t)nline_tab * nz + 1);
    C.EbfTf = C.nbf ? Lo.take<float>(kfz) : nullptr;
  } else {
    C.Vf = C.Bnuf = C.Ebff = C.VTf = C.EbfTf = C.ECf = nullptr;
  }
  if (C.vel) {
    C.vlos = Lo.take<double>(nz);
    C.VR = Lo.take<double>((size_t)C.nray * nline_tab * nz + 1);
    C.VRT = Lo.take<double>((size_t)C.nray * nline_tab * nz + 1);
    // per ray: the Newton-mode derivatives [nnu][zp], or a tangent
    // product's I' [nz][fp]
    C.DXR = Lo.take<double>((size_t)C.nray * std::max(kfz, kfp));
    C.DER = Lo.take<double>((size_t)C.nray * std::max(kfz, kfp));
  } else {
    C.vlos = C.VR = C.VRT = nullptr;
    C.DXR = C.DER = nullptr;
  }
  C.coef = Lo.take<double>((size_t)nz * ncoef(ntr));
  C.ritem = Lo.take<RItem>(std::max(C.nritem, 1));
  C.pitem = Lo.take<PItem>(std::max(C.npitem, 1));
  C.pg_ptr = Lo.take<int>(L * L + 1);
  C.pg_code = Lo.take<int>(4 * ntr + 4 * std::max(C.nment, 1));
  C.eval_n = Lo.take<double>(N);
  C.F = Lo.take<double>(N);
  C.G = Lo.take<double>(N);
  C.Jdag = Lo.take<double>(kf);
  C.JT = Lo.take<double>(kfz);
  C.Jm = Lo.take<double>(kfp);
  C.XS = Lo.take<double>(2 * kfp);
  C.Dchi = Lo.take<double>(kfp);
  C.Deta = Lo.take<double>(kfp);
  C.DchiT = Lo.take<double>(kfz);
  C.DetaT = Lo.take<double>(kfz);
  C.RJ = Lo.take<double>((size_t)nz * std::max(C.nrseg, 1) * 2);
  C.M = Lo.take<double>((size_t)nz * std::max(C.nment, 1) * 2);
  C.P = Lo.take<double>((size_t)nz * L * L);
  C.LU = Lo.take<double>((size_t)nz * L * L);
  C.Fsave = Lo.take<double>(nz);
  C.Gsave = Lo.take<double>(nz);
  C.Psave = Lo.take<double>((size_t)nz * L);
  C.R = Lo.take<double>((size_t)nz * ntr * 2);
  C.Rtot = Lo.take<double>((size_t)nz * ntr * 2);
  C.rho_k = Lo.take<double>(nz);
  C.rows = Lo.take<int>(nz);
  C.rows_frozen = Lo.take<int>(nz);
  C.piv = Lo.take<int>((size_t)nz * L);
  C.n = Lo.take<double>(N);
  C.Fn = Lo.take<double>(N);
  C.Vk = Lo.take<double>((size_t)(m_cap + 1) * N);
  C.H = Lo.take<double>((size_t)(m_cap + 1) * m_cap);
  C.cs = Lo.take<double>(m_cap + 1);
  C.sn = Lo.take<double>(m_cap + 1);
  C.gv = Lo.take<double>(m_cap + 1);
  C.xk = Lo.take<double>(N);
  C.w = Lo.take<double>(N);
  C.lam = Lo.take<double>(nz);
  C.n_init = Lo.take<double>(N);
  C.dots = Lo.take<double>(2 * (m_cap + 1));
  *wbase = Lo.take<int>(ntr + 1);
  *lbase = Lo.take<int>(std::max(C.nline, 1) + 1);
  wp->tiles = Lo.take<Tile>(wsz[0]);
  wp->rate = Lo.take<int4>(wsz[1]);
  wp->pb = Lo.take<int2>(std::max(wsz[2], 1));
  *stage = Lo.take<int>(L);
  *bf_ptr = Lo.take<int>(C.nbf + 1);
  // raw setup inputs (doubles): E, g, A_ul, a_damp, bf_nu, bf_alpha, C_up, w_nu
  *raw = Lo.take<double>(2 * L + 2 * std::max(C.nline, 1) + 2 * std::max(nbf_tot, 1) + (size_t)nz * ntr +
                         nnu);
  (void)in;
}

namespace {
// Everything column creation computes on the host before it touches the
// device (plan_column), kept for the upload (nlte_column_create).
struct ColumnPlan {
  ColDev C{};
  std::vector<TrDev> tr;
  std::vector<int> wbase, lbase, ch_ptr, ch_tr, ch_eptr, ch_ed, pg_ptr, pg_code;
  std::vector<double> Blu;
  std::vector<RItem> ritem;
  std::vector<PItem> pitem;
  std::vector<Tile> tiles;
  std::vector<int4> rate_w;
  std::vector<int2> prec_w;
  std::vector<TileGroup> groups;
  int nline_tab = 0, nbf_tot = 0, nentries = 1, nentries_e = 1, m_cap = 32, nrate0_w = 0;
  int wsz[3] = {0, 0, 0};
  size_t bytes = 0;
};
}  // namespace

// Host half of column creation: validates the descriptors and builds every
// host-side table of the column (transitions, chunk and piece lists, gather
// lists of the preconditioner blocks, single-column work lists) and the size
// of its device arena, with no device call.
static nlte_status plan_column(const nlte_atmos_desc* A, const nlte_atom_desc* M,
                               const nlte_grid_desc* G, const double* C_up, int32_t prec_arg,
                               ColumnPlan& P) {
  const int prec = prec_arg & ~NLTE_DEPTH_SCAN;
  const int scan = (prec_arg & NLTE_DEPTH_SCAN) != 0;
  if (prec != NLTE_FP64 && prec != NLTE_FP32_FORM) return set_err(NLTE_E_INVALID, "bad precision");
  if (scan && A && A->nz > kScanThreads)
    return set_err(NLTE_E_INVALID, "the depth-parallel formal solution takes at most %d depths",
                   kScanThreads);
  if (A && A->vlos && scan)
    return set_err(NLTE_E_INVALID, "columns with a velocity field use the sequential formal solution");
  nlte_status vs = validate(A, M, G, C_up);
  if (vs != NLTE_OK) return vs;

  const int nz = A->nz, L = M->nlev, nline = M->nline, nbf = M->nbf, ntr = nline + nbf;
  const int nnu = G->nnu, nmu = G->nmu;
  P = ColumnPlan{};
  ColDev& C = P.C;
  C.nz = nz; C.L = L; C.ntr = ntr; C.nline = nline; C.nbf = nbf; C.nnu = nnu; C.nmu = nmu;
  C.prec = prec; C.N = nz * L;
  C.scan = scan;
  C.nchunk = (nnu + kWave - 1) / kWave;
  C.fp = C.nchunk * kWave;
  C.zp = (nz + 15) & ~15;
  C.bg_eta = A->eta_c != nullptr;
  C.vel = A->vlos != nullptr;
  C.nray = 2 * nmu;
  C.has_sca = 0;
  if (A->chi_sca)
    for (int k = 0; k < nz; ++k)
      if (A->chi_sca[k] != 0.0) C.has_sca = 1;
  for (int m = 0; m < kMaxMu; ++m) {
    C.wm2[m] = m < nmu ? 0.5 * G->w_mu[m] : 0.0;
    C.inv2mu[m] = m < nmu ? 0.5 / G->mu[m] : 0.0;
    C.wm2f[m] = (float)C.wm2[m];
    C.inv2muf[m] = (float)C.inv2mu[m];
  }
  // transitions, windows, chunk lists
  std::vector<TrDev>& tr = P.tr;
  tr.assign(ntr, TrDev{});
  std::vector<int>& wbase = P.wbase;
  std::vector<int>& lbase = P.lbase;
  wbase.assign(ntr + 1, 0);
  lbase.assign(std::max(nline, 1) + 1, 0);
  int& nline_tab = P.nline_tab;
  std::vector<double>& Blu = P.Blu;
  Blu.assign(nline, 0.0);
  for (int t = 0; t < ntr; ++t) {
    TrDev& T = tr[t];
    T.lo = t < nline ? M->line_lo[t] : M->bf_lo[t - nline];
    T.up = t < nline ? M->line_up[t] : L - 1;
    T.wlo = G->win_lo[t];
    T.whi = G->win_hi[t];
    const int wl = T.whi - T.wlo;
    wbase[t + 1] = wbase[t] + wl;
    T.cwoff = wbase[t];
    if (t < nline) {
      const double nu0 = (M->E[T.up] - M->E[T.lo]) / kH;
      const double Bul = M->A_ul[t] * kC * kC / (2.0 * kH * nu0 * nu0 * nu0);
      T.Blu = M->g[T.up] / M->g[T.lo] * Bul;
      T.g = M->g[T.lo] / M->g[T.up];
      Blu[t] = T.Blu;
      lbase[t + 1] = lbase[t] + wl;
      nline_tab += wl;
    } else {
      T.Blu = 0;
      T.g = 0;
    }
  }
  // V offsets: line tables first ([nz][wl] each), then edge tables ([wl])
  {
    size_t off = 0;
    for (int t = 0; t < nline; ++t) {
      tr[t].voff = (int)off;
      off += (size_t)nz * (tr[t].whi - tr[t].wlo);
    }
    for (int t = nline; t < ntr; ++t) {
      tr[t].voff = (int)off;
      off += tr[t].whi - tr[t].wlo;
    }
    if (off > 0x7fffffff) return set_err(NLTE_E_INVALID, "profile tables too large");
  }

  std::vector<int>& ch_ptr = P.ch_ptr;
  std::vector<int>& ch_tr = P.ch_tr;
  ch_ptr.assign(C.nchunk + 1, 0);
  for (int c = 0; c < C.nchunk; ++c) {
    const int f0 = c * kWave, f1 = std::min(nnu, f0 + kWave);
    for (int t = 0; t < nline; ++t)
      if (tr[t].wlo < f1 && tr[t].whi > f0) ch_tr.push_back(t);
    ch_ptr[c + 1] = (int)ch_tr.size();
  }
  std::vector<int>& ch_eptr = P.ch_eptr;
  std::vector<int>& ch_ed = P.ch_ed;
  ch_eptr.assign(C.nchunk + 1, 0);
  for (int c = 0; c < C.nchunk; ++c) {
    const int f0 = c * kWave, f1 = std::min(nnu, f0 + kWave);
    for (int t = nline; t < ntr; ++t)
      if (tr[t].wlo < f1 && tr[t].whi > f0) ch_ed.push_back(t);
    ch_eptr[c + 1] = (int)ch_ed.size();
  }
  // pieces of the frequency axis: cut at every window edge (and into at most
  // seg_len frequencies), so that each piece lies inside or outside every
  // window.  The rate integrals of the s transitions covering a piece run as
  // blocks of up to kRateBlk lines and kRateBlk edges; the pair sums give the
  // piece s^2 entries (t, t') and run as blocks of at most kPairBlk^2 of them
  // velocity-field columns take the shortest pieces, since their pair sums
  // walk every ray at every frequency (512-column velocity batch: 1410 ms
  // per solve with pieces of 512, 1064 with 96, 989 with 32, 982 with 16,
  // whose extra entries slow the assembly)
  constexpr int kSegLenVel = 32;
  const int seg_len = scan ? kSegLenScan : C.vel ? kSegLenVel : kSegLen;
  std::vector<int> cuts;
  for (int t = 0; t < ntr; ++t) {
    cuts.push_back(tr[t].wlo);
    cuts.push_back(tr[t].whi);
  }
  std::sort(cuts.begin(), cuts.end());
  cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
  std::vector<PItem>& pitem = P.pitem;
  std::vector<RItem>& ritem = P.ritem;
  std::vector<int2> ment;  // (t, t') of each entry
  std::vector<int> rcount(ntr, 0);  // rate entries per transition so far
  for (size_t c = 0; c + 1 < cuts.size(); ++c) {
    std::vector<int> A;
    for (int t = 0; t < ntr; ++t)
      if (tr[t].wlo <= cuts[c] && tr[t].whi >= cuts[c + 1]) A.push_back(t);
    const int s = (int)A.size();
    for (int a = cuts[c]; s > 0 && a < cuts[c + 1]; a += seg_len) {
      const int b = std::min(a + seg_len, cuts[c + 1]);
      // rate blocks: lines and edges of A (A is sorted, lines first); the
      // line rates of velocity-field columns come from their formal-solution
      // kernel (entries per chunk, below)
      std::vector<int> Ln, Ed;
      for (int t : A) (t < nline ? Ln : Ed).push_back(t);
      if (C.vel) Ln.clear();
      for (size_t li = 0, ei = 0; li < Ln.size() || ei < Ed.size();) {
        RItem R{};
        R.f0 = a;
        R.f1 = b;
        R.nl = (int)std::min<size_t>(kRateBlk, Ln.size() - li);
        R.ne = (int)std::min<size_t>(kRateBlk, Ed.size() - ei);
        for (int i = 0; i < R.nl; ++i) R.t[i] = Ln[li + i];
        for (int i = 0; i < R.ne; ++i) R.t[R.nl + i] = Ed[ei + i];
        for (int i = 0; i < R.nl + R.ne; ++i) R.e[i] = rcount[R.t[i]]++;  // ordinal, offset below
        li += R.nl;
        ei += R.ne;
        ritem.push_back(R);
      }
      const int e0 = (int)ment.size();
      for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) ment.push_back(make_int2(A[i], A[j]));
      for (int ti = 0; ti < s; ti += kPairBlk)
        for (int ui = 0; ui < s; ui += kPairBlk) {
          PItem P{};
          P.f0 = a;
          P.f1 = b;
          P.nt = std::min(kPairBlk, s - ti);
          P.nu = std::min(kPairBlk, s - ui);
          P.e0 = e0 + ti * s + ui;
          P.es = s;
          P.same = ti == ui;
          for (int i = 0; i < P.nt; ++i) P.t[i] = A[ti + i];
          for (int j = 0; j < P.nu; ++j) P.u[j] = A[ui + j];
          pitem.push_back(P);
        }
    }
  }
  C.npitem = (int)pitem.size();
  C.nment = (int)ment.size();
  // rate entries: transition by transition, each in frequency order;
  // velocity-field columns: one per 64-frequency chunk a line's window meets
  if (C.vel)
    for (int t = 0; t < nline; ++t) rcount[t] = (tr[t].whi - 1) / kWave - tr[t].wlo / kWave + 1;
  {
    int first = 0;
    for (int t = 0; t < ntr; ++t) {
      tr[t].sfirst = first;
      tr[t].nseg = rcount[t];
      first += rcount[t];
    }
    for (RItem& R : ritem)
      for (int i = 0; i < R.nl + R.ne; ++i) R.e[i] += tr[R.t[i]].sfirst;
    C.nrseg = first;
    C.nritem = (int)ritem.size();
  }
  // gather lists of the preconditioner blocks: entry (i, j) sums
  //   Gamma: (lo,lo) += C_lu+R_lu, (up,up) += C_ul+R_ul, (lo,up) -= C_ul+R_ul, (up,lo) -= C_lu+R_lu
  //   entries: (lo_t,lo_u) += M1, (up_t,lo_u) -= M1, (lo_t,up_u) += M2, (up_t,up_u) -= M2
  // code = (index << 3) | (kind << 1) | negate; kind 0/1: total up/down rate, 2/3: M1/M2
  std::vector<std::vector<int>> gl(L * L);
  for (int t = 0; t < ntr; ++t) {
    const int lo = tr[t].lo, up = tr[t].up;
    gl[lo * L + lo].push_back((t << 3) | (0 << 1) | 0);
    gl[up * L + up].push_back((t << 3) | (1 << 1) | 0);
    gl[lo * L + up].push_back((t << 3) | (1 << 1) | 1);
    gl[up * L + lo].push_back((t << 3) | (0 << 1) | 1);
  }
  for (int q = 0; q < C.nment; ++q) {
    const TrDev& Tt = tr[ment[q].x];
    const TrDev& Tu = tr[ment[q].y];
    gl[Tt.lo * L + Tu.lo].push_back((q << 3) | (2 << 1) | 0);
    gl[Tt.up * L + Tu.lo].push_back((q << 3) | (2 << 1) | 1);
    gl[Tt.lo * L + Tu.up].push_back((q << 3) | (3 << 1) | 0);
    gl[Tt.up * L + Tu.up].push_back((q << 3) | (3 << 1) | 1);
  }
  std::vector<int>& pg_ptr = P.pg_ptr;
  std::vector<int>& pg_code = P.pg_code;
  pg_ptr.assign(L * L + 1, 0);
  for (int e = 0; e < L * L; ++e) {
    pg_code.insert(pg_code.end(), gl[e].begin(), gl[e].end());
    pg_ptr[e + 1] = (int)pg_code.size();
  }
  P.nentries = std::max<int>(1, (int)ch_tr.size());
  P.nentries_e = std::max<int>(1, (int)ch_ed.size());
  P.nbf_tot = nbf ? M->bf_ptr[nbf] : 0;
  P.m_cap = 32;

  // single-column work lists
  int maxL_w = 0;
  P.nrate0_w = build_work_lists(&C, 1, P.tiles, P.groups, P.rate_w, P.prec_w, maxL_w);
  P.wsz[0] = (int)P.tiles.size();
  P.wsz[1] = (int)P.rate_w.size();
  P.wsz[2] = (int)P.prec_w.size();

  // size of the device arena
  SetupIn in{};
  TrDev* tr_d;
  int *wbase_d, *lbase_d, *stage_d, *bfptr_d;
  WorkPtrs wp{};
  double* raw_d;
  Layout sizer(nullptr);
  ColDev tmp = C;
  layout_column(sizer, tmp, in, wbase[ntr], nline_tab, P.nbf_tot, P.nentries, P.nentries_e, P.m_cap,
                &tr_d, &wbase_d, &lbase_d, &wp, P.wsz, &stage_d, &bfptr_d, &raw_d);
  P.bytes = sizer.off + 256;
  return NLTE_OK;
}

// Bytes of a pooled arena for a column of `plan` arena bytes: the arena,
// then its device descriptor.
size_t nlte::pooled_arena_bytes(size_t plan) {
  return ((plan + 255) / 256) * 256 + ((sizeof(ColDev) + 255) / 256) * 256;
}

static nlte_status column_create_impl(nlte_ctx* ctx, const nlte_atmos_desc* A,
                                      const nlte_atom_desc* M, const nlte_grid_desc* G,
                                      const double* C_up, int32_t prec_arg, hipStream_t stream,
                                      void* pool_arena, size_t pool_cap, nlte_column** out);

extern "C" nlte_status nlte_column_create(nlte_ctx* ctx, const nlte_atmos_desc* A,
                                          const nlte_atom_desc* M, const nlte_grid_desc* G,
                                          const double* C_up, int32_t prec_arg,
                                          hipStream_t stream, nlte_column** out) {
  return column_create_impl(ctx, A, M, G, C_up, prec_arg, stream, nullptr, 0, out);
}

// pool_arena (NULL: the column allocates its own) holds pool_cap bytes, at
// least pooled_arena_bytes(plan) of them; the column lays itself out at its
// start, puts its device descriptor after it, and never frees it.
static nlte_status column_create_impl(nlte_ctx* ctx, const nlte_atmos_desc* A,
                                      const nlte_atom_desc* M, const nlte_grid_desc* G,
                                      const double* C_up, int32_t prec_arg, hipStream_t stream,
                                      void* pool_arena, size_t pool_cap, nlte_column** out) {
  if (!ctx || !out) return set_err(NLTE_E_INVALID, "NULL ctx/out");
  // an error left pending by an unrelated earlier call stays pending for its
  // owner (peeked, not cleared); the setup launches are judged by whether
  // they leave a different one
  const hipError_t pending = hipPeekAtLastError();
  ColumnPlan P;
  const nlte_status ps = plan_column(A, M, G, C_up, prec_arg, P);
  if (ps != NLTE_OK) return ps;
  HIP_TRY(hipSetDevice(ctx->device));
  ColDev& C = P.C;
  const int nz = C.nz, L = C.L, nline = C.nline, nbf = C.nbf, ntr = C.ntr, nnu = C.nnu;
  const int prec = C.prec;
  const std::vector<TrDev>& tr = P.tr;
  const std::vector<int>& wbase = P.wbase;
  const std::vector<int>& lbase = P.lbase;
  const int nline_tab = P.nline_tab, nbf_tot = P.nbf_tot;
  const int* wsz = P.wsz;
  const std::vector<int>&ch_ptr = P.ch_ptr, &ch_tr = P.ch_tr, &ch_eptr = P.ch_eptr, &ch_ed = P.ch_ed;
  const std::vector<RItem>& ritem = P.ritem;
  const std::vector<PItem>& pitem = P.pitem;
  const std::vector<int>&pg_ptr = P.pg_ptr, &pg_code = P.pg_code;
  const std::vector<Tile>& tiles = P.tiles;
  const std::vector<int4>& rate_w = P.rate_w;
  const std::vector<int2>& prec_w = P.prec_w;
  const std::vector<TileGroup>& groups = P.groups;
  const int nrate0_w = P.nrate0_w;
  nlte_column* col = new nlte_column();
  col->ctx = ctx;
  col->device = ctx->device;
  col->arena_bytes = P.bytes;
  if (pool_arena) {
    if (pool_cap < pooled_arena_bytes(P.bytes)) {
      delete col;
      return set_err(NLTE_E_INVALID, "pooled arena of %zu bytes for a column of %zu", pool_cap,
                     P.bytes);
    }
    col->pooled = true;
    col->arena = pool_arena;
  } else {
    hipError_t he = hipMalloc(&col->arena, col->arena_bytes);
    if (he != hipSuccess) {
      delete col;
      return set_err(NLTE_E_NOMEM, "hipMalloc(%zu) failed: %s", P.bytes, hipGetErrorString(he));
    }
  }
  // the arena goes back to a pool or to the device on every failure below
  auto release = [col]() {
    if (col->pooled) return;
    if (col->d) (void)hipFree(col->d);
    (void)hipFree(col->arena);
  };
  SetupIn in{};
  TrDev* tr_d;
  int *wbase_d, *lbase_d, *stage_d, *bfptr_d;
  WorkPtrs wp{};
  double* raw_d;
  Layout lay(col->arena);
  layout_column(lay, C, in, wbase[ntr], nline_tab, nbf_tot, P.nentries, P.nentries_e, P.m_cap, &tr_d,
                &wbase_d, &lbase_d, &wp, wsz, &stage_d, &bfptr_d, &raw_d);
  col->restart_cap = P.m_cap;
  col->Blu = P.Blu;

  // upload
  auto up = [&](const void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, stream);
  };
  std::vector<double> zeros(nz, 0.0);
  double* rE = raw_d;
  double* rg = rE + L;
  double* rA = rg + L;
  double* ra = rA + std::max(nline, 1);
  double* rbn = ra + std::max(nline, 1);
  double* rba = rbn + std::max(nbf_tot, 1);
  double* rC = rba + std::max(nbf_tot, 1);
  double* rW = rC + (size_t)nz * ntr;
  hipError_t e = hipSuccess;
#define UP(d, s, b) if (e == hipSuccess) e = up(d, s, b)
  UP(C.z, A->z, nz * 8);
  UP(C.T, A->T, nz * 8);
  UP(C.ne, A->ne, nz * 8);
  UP(C.ntot, A->ntot, nz * 8);
  UP(C.chi_c, A->chi_c, nz * 8);
  UP(C.chi_sca, A->chi_sca ? A->chi_sca : zeros.data(), nz * 8);
  UP(C.nu, G->nu, nnu * 8);
  UP(tr_d, tr.data(), ntr * sizeof(TrDev));
  UP(C.ch_lptr, ch_ptr.data(), ch_ptr.size() * 4);
  UP(C.ch_line, ch_tr.data(), ch_tr.size() * 4);
  UP(C.ch_eptr, ch_eptr.data(), ch_eptr.size() * 4);
  UP(C.ch_edge, ch_ed.data(), ch_ed.size() * 4);
  UP(C.ritem, ritem.data(), ritem.size() * sizeof(RItem));
  UP(C.pitem, pitem.data(), pitem.size() * sizeof(PItem));
  UP(wp.rate, rate_w.data(), rate_w.size() * sizeof(int4));
  UP(wp.pb, prec_w.data(), prec_w.size() * sizeof(int2));
  UP(C.pg_ptr, pg_ptr.data(), pg_ptr.size() * 4);
  UP(C.pg_code, pg_code.data(), pg_code.size() * 4);
  UP(wbase_d, wbase.data(), wbase.size() * 4);
  UP(lbase_d, lbase.data(), lbase.size() * 4);
  UP(wp.tiles, tiles.data(), tiles.size() * sizeof(Tile));
  UP(stage_d, M->stage, L * 4);
  if (nbf) UP(bfptr_d, M->bf_ptr, (nbf + 1) * 4);
  UP(rE, M->E, L * 8);
  UP(rg, M->g, L * 8);
  if (nline) {
    UP(rA, M->A_ul, nline * 8);
    UP(ra, M->a_damp, nline * 8);
  }
  if (nbf_tot) {
    UP(rbn, M->bf_nu, nbf_tot * 8);
    UP(rba, M->bf_alpha, nbf_tot * 8);
  }
  UP(rC, C_up, (size_t)nz * ntr * 8);
  if (G->w_nu) UP(rW, G->w_nu, (size_t)nnu * 8);
  if (A->eta_c) UP(C.EC, A->eta_c, (size_t)nz * nnu * 8);
  if (A->vlos) UP(C.vlos, A->vlos, (size_t)nz * 8);
#undef UP
  if (e == hipSuccess) e = hipMemsetAsync(C.st, 0, sizeof(ColState), stream);
  if (e != hipSuccess) {
    release();
    delete col;
    return set_err(NLTE_E_DEVICE, "upload failed: %s", hipGetErrorString(e));
  }
  in.E = rE; in.g = rg; in.A_ul = rA; in.a_damp = ra; in.bf_nu = rbn; in.bf_alpha = rba; in.C_up = rC;
  in.w_nu = G->w_nu ? rW : nullptr;
  in.stage = stage_d; in.bf_ptr = bfptr_d; in.mass_amu = M->mass_amu; in.vturb = M->vturb;
  for (int m = 0; m < kMaxMu; ++m) in.mu[m] = m < G->nmu ? G->mu[m] : 0.0;

  // setup kernels
  k_setup_depth<<<(nz + 63) / 64, 64, 0, stream>>>(C, in);
  {
    const size_t n = (size_t)nz * nnu;
    k_setup_freq<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(C);
  }
  k_setup_window<<<(wbase[ntr] + 255) / 256, 256, 0, stream>>>(C, in, wbase_d, wbase[ntr]);
  if (nline) {
    const size_t n = (size_t)lbase[nline] * nz;
    k_setup_voigt<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(C, in, lbase_d, lbase[nline]);
  }
  k_setup_norm<<<(ntr * nz + 63) / 64, 64, 0, stream>>>(C, in);
  if (C.vel && nline) {
    const size_t n = (size_t)lbase[nline] * nz * C.nray;
    k_setup_voigt_vel<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(C, in, lbase_d, lbase[nline]);
    k_setup_norm_vel<<<(nline * C.nray * nz + 63) / 64, 64, 0, stream>>>(C, in);
    k_setup_rsp_vel<<<(nline * nz + 63) / 64, 64, 0, stream>>>(C);
    const size_t nvr = (size_t)C.nray * nline_tab * nz;
    k_setup_transpose_vel<<<(unsigned)((nvr + 255) / 256), 256, 0, stream>>>(C, nvr);
  }
  {
    const size_t n = std::max((size_t)nz * nnu, (size_t)nline_tab * nz);
    k_setup_transpose<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(C, nline_tab * nz);
  }
  if (prec == NLTE_FP32_FORM) {
    const size_t nv = (size_t)nline_tab * nz + (wbase[ntr] - nline_tab);
    const size_t nvt = (size_t)nline_tab * nz;
    const size_t n = std::max(nv, (size_t)nz * nnu);
    k_setup_f32<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(C, nv, nvt);
  }
  e = hipPeekAtLastError();
  if (e == pending) e = hipSuccess;  // nothing new from the setup launches
  else (void)hipGetLastError();     // the setup's own launch error, reported below
  if (e == hipSuccess) {
    if (col->pooled)
      col->d = reinterpret_cast<ColDev*>(static_cast<char*>(col->arena) + ((P.bytes + 255) / 256) * 256);
    else
      e = hipMalloc(&col->d, sizeof(ColDev));
  }
  if (e == hipSuccess) e = hipMemcpyAsync(col->d, &C, sizeof(ColDev), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    release();
    delete col;
    return set_err(NLTE_E_DEVICE, "column setup failed: %s", hipGetErrorString(e));
  }
  col->h = C;
  col->bw.cols = col->d;
  col->bw.tiles = wp.tiles;
  col->bw.rate_work = wp.rate;
  col->bw.pb_work = wp.pb;
  col->bw.ncol = 1;
  col->bw.ntiles = wsz[0];
  col->bw.nrate = wsz[1];
  col->bw.nrate0 = nrate0_w;
  col->bw.npb = wsz[2];
  col->bw.any64 = prec == NLTE_FP64;
  col->bw.any32 = prec == NLTE_FP32_FORM;
  col->bw.any_newton = 1;
  set_groups(col->bw, groups);  // one column: at most one group
  col->bw.maxnz = nz;

  *out = col;
  return NLTE_OK;
}

extern "C" void nlte_column_destroy(nlte_column* col) {
  if (!col) return;
  (void)hipSetDevice(col->device);
  if (!col->pooled) {
    if (col->d) (void)hipFree(col->d);
    if (col->arena) (void)hipFree(col->arena);
  }
  delete col;
}

// ---------------------------------------------------------------------------
// problems held on the host until their column is created (served requests)
// ---------------------------------------------------------------------------
namespace nlte {
struct HostProblem {
  std::vector<double> z, T, ne, ntot, chi_c, chi_sca, eta_c, vlos;
  std::vector<double> E, g, A_ul, a_damp, bf_nu, bf_alpha;
  std::vector<int32_t> stage, line_lo, line_up, bf_lo, bf_ptr;
  std::vector<double> nu, mu, w_mu, w_nu, C_up;
  std::vector<int32_t> win_lo, win_hi;
  nlte_atmos_desc A{};
  nlte_atom_desc M{};
  nlte_grid_desc G{};
  int32_t precision = 0;
  size_t bytes = 0;
};

template <typename T>
static void copy_in(std::vector<T>& v, const T* p, size_t n) {
  if (p) v.assign(p, p + n);
}
template <typename T>
static const T* ptr_or_null(const std::vector<T>& v) {
  return v.empty() ? nullptr : v.data();
}

// Validates and sizes a problem (as nlte_column_plan_bytes), then copies
// every descriptor array, so the caller may free its own right away.
nlte_status problem_copy(const nlte_atmos_desc* A, const nlte_atom_desc* M, const nlte_grid_desc* G,
                         const double* C_up, int32_t precision, HostProblem** out) {
  ColumnPlan P;
  const nlte_status st = plan_column(A, M, G, C_up, precision, P);
  if (st != NLTE_OK) return st;
  HostProblem* H = new HostProblem();
  const int nz = A->nz, L = M->nlev, nline = M->nline, nbf = M->nbf, ntr = nline + nbf;
  const int nnu = G->nnu, nmu = G->nmu;
  const size_t nbft = nbf ? (size_t)M->bf_ptr[nbf] : 0;
  copy_in(H->z, A->z, nz); copy_in(H->T, A->T, nz); copy_in(H->ne, A->ne, nz);
  copy_in(H->ntot, A->ntot, nz); copy_in(H->chi_c, A->chi_c, nz);
  copy_in(H->chi_sca, A->chi_sca, nz); copy_in(H->eta_c, A->eta_c, (size_t)nz * nnu);
  copy_in(H->vlos, A->vlos, nz);
  copy_in(H->E, M->E, L); copy_in(H->g, M->g, L); copy_in(H->stage, M->stage, L);
  copy_in(H->line_lo, M->line_lo, nline); copy_in(H->line_up, M->line_up, nline);
  copy_in(H->A_ul, M->A_ul, nline); copy_in(H->a_damp, M->a_damp, nline);
  copy_in(H->bf_lo, M->bf_lo, nbf);
  if (nbf) copy_in(H->bf_ptr, M->bf_ptr, nbf + 1);
  copy_in(H->bf_nu, M->bf_nu, nbft); copy_in(H->bf_alpha, M->bf_alpha, nbft);
  copy_in(H->nu, G->nu, nnu); copy_in(H->win_lo, G->win_lo, ntr); copy_in(H->win_hi, G->win_hi, ntr);
  copy_in(H->mu, G->mu, nmu); copy_in(H->w_mu, G->w_mu, nmu); copy_in(H->w_nu, G->w_nu, nnu);
  copy_in(H->C_up, C_up, (size_t)nz * ntr);
  H->A = nlte_atmos_desc{nz, H->z.data(), H->T.data(), H->ne.data(), H->ntot.data(), H->chi_c.data(),
                         ptr_or_null(H->chi_sca), ptr_or_null(H->eta_c), ptr_or_null(H->vlos)};
  H->M = nlte_atom_desc{L, H->E.data(), H->g.data(), H->stage.data(), nline, ptr_or_null(H->line_lo),
                        ptr_or_null(H->line_up), ptr_or_null(H->A_ul), ptr_or_null(H->a_damp),
                        M->mass_amu, M->vturb, nbf, ptr_or_null(H->bf_lo), ptr_or_null(H->bf_ptr),
                        ptr_or_null(H->bf_nu), ptr_or_null(H->bf_alpha)};
  H->G = nlte_grid_desc{nnu, H->nu.data(), H->win_lo.data(), H->win_hi.data(), nmu, H->mu.data(),
                        H->w_mu.data(), ptr_or_null(H->w_nu)};
  H->precision = precision;
  H->bytes = P.bytes;
  *out = H;
  return NLTE_OK;
}

size_t problem_bytes(const HostProblem* H) { return H->bytes; }

nlte_status problem_create_column(nlte_ctx* ctx, const HostProblem* H, hipStream_t s,
                                  void* pool_arena, size_t pool_cap, nlte_column** out) {
  return column_create_impl(ctx, &H->A, &H->M, &H->G, H->C_up.data(), H->precision, s,
                            pool_arena, pool_cap, out);
}

void problem_free(HostProblem* H) { delete H; }
}  // namespace nlte

extern "C" nlte_status nlte_column_plan_bytes(const nlte_atmos_desc* atmos,
                                              const nlte_atom_desc* atom,
                                              const nlte_grid_desc* grid, const double* C_up,
                                              int32_t precision, size_t* bytes) {
  if (!bytes) return set_err(NLTE_E_INVALID, "bytes is NULL");
  ColumnPlan P;
  const nlte_status st = plan_column(atmos, atom, grid, C_up, precision, P);
  if (st != NLTE_OK) return st;
  *bytes = P.bytes;
  return NLTE_OK;
}

extern "C" nlte_status nlte_column_bytes(const nlte_column* col, size_t* bytes) {
  if (!col || !bytes) return set_err(NLTE_E_INVALID, "NULL argument");
  *bytes = col->arena_bytes;
  return NLTE_OK;
}

extern "C" nlte_status nlte_column_dims(const nlte_column* col, int32_t dims[8]) {
  if (!col || !dims) return set_err(NLTE_E_INVALID, "NULL argument");
  const ColDev& C = col->h;
  dims[0] = C.nz; dims[1] = C.L; dims[2] = C.ntr; dims[3] = C.nline;
  dims[4] = C.nbf; dims[5] = C.nnu; dims[6] = C.nmu; dims[7] = C.prec | (C.scan ? NLTE_DEPTH_SCAN : 0);
  return NLTE_OK;
}

// ---------------------------------------------------------------------------
// small vector kernels for the API entry points
// ---------------------------------------------------------------------------
__global__ void k_axpy_into(double* __restrict__ y, const double* __restrict__ x,
                            const double* __restrict__ v, double a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] + a * v[i];
}

__global__ void k_diff_scaled(double* __restrict__ out, const double* __restrict__ F1,
                              const double* __restrict__ F0, double inv_eps, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (F1[i] - F0[i]) * inv_eps;
}

__global__ void k_jbar(double* __restrict__ out, const double* __restrict__ R,
                       const TrDev* __restrict__ tr, int nz, int ntr, int nline) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nz * nline) return;
  const int k = i / nline, t = i % nline;
  out[i] = R[((size_t)k * ntr + t) * 2] / tr[t].Blu;
}

__global__ void k_check_finite_pos(const double* __restrict__ n, int N, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) {
    const double v = n[i];
    if (!(v > 0.0) || !isfinite(v)) atomicOr(flag, 1);
  }
}

__global__ void k_set_eval(ColState* st, int mode, int want_J, int rows_own, int prec) {
  st->mode = mode;
  st->want_J = want_J;
  st->rows_own = rows_own;
  st->cur_prec = prec;
}

namespace nlte {
hipError_t set_state_eval(nlte_column* col, int mode, int want_J, int rows_own, hipStream_t s) {
  k_set_eval<<<1, 1, 0, s>>>(col->h.st, mode, want_J, rows_own, col->h.prec);
  return hipGetLastError();
}
}  // namespace nlte

static nlte_status run_single(nlte_column* col, hipStream_t s) {
  const ColDev& C = col->h;
  (void)C;
  HIP_TRY(launch_residual(col->bw, s));
  return NLTE_OK;
}

static nlte_status check_populations(nlte_column* col, const double* n_dev, hipStream_t s) {
  int* flag = nullptr;
  HIP_TRY(hipMallocAsync((void**)&flag, sizeof(int), s));
  int h = 0;
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e == hipSuccess) {
    k_check_finite_pos<<<(col->h.N + 255) / 256, 256, 0, s>>>(n_dev, col->h.N, flag);
    e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFreeAsync(flag, s);
  if (e != hipSuccess) return set_err(NLTE_E_DEVICE, "population check failed: %s", hipGetErrorString(e));
  if (h) return set_err(NLTE_E_NONFINITE, "populations must be finite and positive");
  return NLTE_OK;
}

extern "C" nlte_status nlte_lte_populations(nlte_column* col, double* n_dev, hipStream_t s) {
  if (!col || !n_dev) return set_err(NLTE_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(col->ctx->device));
  HIP_TRY(hipMemcpyAsync(n_dev, col->h.nstar, col->h.N * 8, hipMemcpyDeviceToDevice, s));
  return NLTE_OK;
}

extern "C" nlte_status nlte_residual(nlte_column* col, const double* n_dev, double* F_dev,
                                     double* J_dev, double* R_dev, double* Jbar_dev,
                                     double* P_dev, int update_J, hipStream_t s) {
  if (!col || !n_dev || !F_dev) return set_err(NLTE_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(col->ctx->device));
  nlte_status st = check_populations(col, n_dev, s);
  if (st != NLTE_OK) return st;
  const ColDev& C = col->h;
  const int newton = P_dev != nullptr;
  const int wantJ = (J_dev != nullptr) || update_J;
  HIP_TRY(hipMemcpyAsync(C.eval_n, n_dev, C.N * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(set_state_eval(col, newton ? kModeNewton : kModeF, wantJ, 1, s));
  st = run_single(col, s);
  if (st != NLTE_OK) return st;
  HIP_TRY(hipMemcpyAsync(F_dev, C.F, C.N * 8, hipMemcpyDeviceToDevice, s));
  if (J_dev) transpose_J(C, J_dev, s);
  if (update_J) transpose_J(C, C.Jdag, s);
  if (R_dev) HIP_TRY(hipMemcpyAsync(R_dev, C.R, (size_t)C.nz * C.ntr * 16, hipMemcpyDeviceToDevice, s));
  if (Jbar_dev && C.nline)
    k_jbar<<<(C.nz * C.nline + 255) / 256, 256, 0, s>>>(Jbar_dev, C.R, C.tr, C.nz, C.ntr, C.nline);
  if (P_dev) HIP_TRY(hipMemcpyAsync(P_dev, C.P, (size_t)C.nz * C.L * C.L * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(set_state_eval(col, kModeIdle, 0, 0, s));
  HIP_TRY(hipGetLastError());
  return NLTE_OK;
}

// Scratch layout of one allocation-free residual evaluation: the column's
// descriptor, the population-check flag, the level coefficients and the
// formal-solution, rate and pair-sum scratch (the buffers the column's own
// evaluations keep in its arena).  Returns the bytes needed.
static size_t noalloc_layout(const ColDev& H, char* base, ColDev* C, int** flag, ColDev** dcol) {
  Layout Lo(base);
  const size_t kfp = (size_t)H.nz * H.fp, kfz = (size_t)H.nnu * H.zp;
  *dcol = Lo.take<ColDev>(1);
  *flag = Lo.take<int>(1);
  C->coef = Lo.take<double>((size_t)H.nz * ncoef(H.ntr));
  C->Jm = Lo.take<double>(kfp);
  C->XS = Lo.take<double>(2 * kfp);
  C->Dchi = Lo.take<double>(kfp);
  C->Deta = Lo.take<double>(kfp);
  C->JT = Lo.take<double>(kfz);
  C->DchiT = Lo.take<double>(kfz);
  C->DetaT = Lo.take<double>(kfz);
  C->RJ = Lo.take<double>((size_t)H.nz * std::max(H.nrseg, 1) * 2);
  C->M = Lo.take<double>((size_t)H.nz * std::max(H.nment, 1) * 2);
  if (H.vel) {  // per-ray local intensity derivatives of velocity-field columns
    C->DXR = Lo.take<double>((size_t)H.nray * kfz);
    C->DER = Lo.take<double>((size_t)H.nray * kfz);
  }
  return Lo.off;
}

__global__ void k_put_coldev(ColDev c, ColDev* dst) { *dst = c; }
__global__ void k_zero_int(int* p) { *p = 0; }

extern "C" nlte_status nlte_residual_noalloc(nlte_column* col, const double* n_dev, double* F_dev,
                                             double* J_dev, double* R_dev, double* Jbar_dev,
                                             double* P_dev, int update_J, hipStream_t s) {
  if (!col || !n_dev || !F_dev) return set_err(NLTE_E_INVALID, "NULL argument");
  const ColDev& H = col->h;
  ColDev C = H;
  int* flag = nullptr;
  ColDev* dcol = nullptr;
  const size_t need = noalloc_layout(H, nullptr, &C, &flag, &dcol);
  if (need > kScratchBytes)
    return set_err(NLTE_E_INVALID,
                   "column needs %zu bytes of evaluation scratch; the allocation-free entry point "
                   "holds %zu",
                   need, kScratchBytes);
  HIP_TRY(hipSetDevice(col->device));
  hipError_t se = hipSuccess;
  char* base = scratch_base(col->device, &se);
  if (!base) return set_err(NLTE_E_DEVICE, "scratch address lookup failed: %s", hipGetErrorString(se));
  noalloc_layout(H, base, &C, &flag, &dcol);
  k_put_coldev<<<1, 1, 0, s>>>(C, dcol);
  // populations positive and finite (flag in the scratch, cleared first)
  k_zero_int<<<1, 1, 0, s>>>(flag);
  k_check_finite_pos<<<(H.N + 255) / 256, 256, 0, s>>>(n_dev, H.N, flag);
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h) return set_err(NLTE_E_NONFINITE, "populations must be finite and positive");
  const int newton = P_dev != nullptr;
  const int wantJ = (J_dev != nullptr) || update_J;
  HIP_TRY(hipMemcpyAsync(H.eval_n, n_dev, H.N * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(set_state_eval(col, newton ? kModeNewton : kModeF, wantJ, 1, s));
  BatchWork bw = col->bw;
  bw.cols = dcol;
  bw.single_stream = 1;
  HIP_TRY(launch_residual(bw, s));
  HIP_TRY(hipMemcpyAsync(F_dev, H.F, H.N * 8, hipMemcpyDeviceToDevice, s));
  if (J_dev) transpose_J(C, J_dev, s);
  if (update_J) transpose_J(C, H.Jdag, s);
  if (R_dev) HIP_TRY(hipMemcpyAsync(R_dev, H.R, (size_t)H.nz * H.ntr * 16, hipMemcpyDeviceToDevice, s));
  if (Jbar_dev && H.nline)
    k_jbar<<<(H.nz * H.nline + 255) / 256, 256, 0, s>>>(Jbar_dev, H.R, H.tr, H.nz, H.ntr, H.nline);
  if (P_dev) HIP_TRY(hipMemcpyAsync(P_dev, H.P, (size_t)H.nz * H.L * H.L * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(set_state_eval(col, kModeIdle, 0, 0, s));
  HIP_TRY(hipGetLastError());
  return NLTE_OK;
}

extern "C" nlte_status nlte_jvp(nlte_column* col, const double* n_dev, const double* v_dev,
                                double eps, double* Jv_dev, hipStream_t s) {
  if (!col || !n_dev || !v_dev || !Jv_dev) return set_err(NLTE_E_INVALID, "NULL argument");
  if (!(eps != 0.0) || !isfinite(eps)) return set_err(NLTE_E_INVALID, "eps must be finite and nonzero");
  HIP_TRY(hipSetDevice(col->ctx->device));
  nlte_status st = check_populations(col, n_dev, s);
  if (st != NLTE_OK) return st;
  const ColDev& C = col->h;
  // F(n) with its own rows, kept in Fn; rows frozen for the perturbed call
  HIP_TRY(hipMemcpyAsync(C.eval_n, n_dev, C.N * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(set_state_eval(col, kModeF, 0, 1, s));
  st = run_single(col, s);
  if (st != NLTE_OK) return st;
  HIP_TRY(hipMemcpyAsync(C.Fn, C.F, C.N * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(C.rows_frozen, C.rows, C.nz * 4, hipMemcpyDeviceToDevice, s));
  k_axpy_into<<<(C.N + 255) / 256, 256, 0, s>>>(C.eval_n, n_dev, v_dev, eps, C.N);
  HIP_TRY(set_state_eval(col, kModeF, 0, 0, s));
  st = run_single(col, s);
  if (st != NLTE_OK) return st;
  k_diff_scaled<<<(C.N + 255) / 256, 256, 0, s>>>(Jv_dev, C.F, C.Fn, 1.0 / eps, C.N);
  HIP_TRY(set_state_eval(col, kModeIdle, 0, 0, s));
  HIP_TRY(hipGetLastError());
  return NLTE_OK;
}

__global__ void k_set_tangent(ColState* st, int on) {
  st->mode = kModeIdle;
  st->tan_pending = on;
}

extern "C" nlte_status nlte_jvp_tangent(nlte_column* col, const double* n_dev, const double* v_dev,
                                        double* Jv_dev, hipStream_t s) {
  if (!col || !n_dev || !v_dev || !Jv_dev) return set_err(NLTE_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(col->ctx->device));
  nlte_status st = check_populations(col, n_dev, s);
  if (st != NLTE_OK) return st;
  const ColDev& C = col->h;
  // rates, total rates and rows of n (its own rows)
  HIP_TRY(hipMemcpyAsync(C.eval_n, n_dev, C.N * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(set_state_eval(col, kModeF, 0, 1, s));
  st = run_single(col, s);
  if (st != NLTE_OK) return st;
  HIP_TRY(hipMemcpyAsync(C.rows_frozen, C.rows, C.nz * 4, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(C.n, n_dev, C.N * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(C.eval_n, v_dev, C.N * 8, hipMemcpyDeviceToDevice, s));
  k_set_tangent<<<1, 1, 0, s>>>(C.st, 1);
  HIP_TRY(launch_tangent(col->bw, s));
  HIP_TRY(hipMemcpyAsync(Jv_dev, C.F, C.N * 8, hipMemcpyDeviceToDevice, s));
  k_set_tangent<<<1, 1, 0, s>>>(C.st, 0);
  HIP_TRY(hipGetLastError());
  return NLTE_OK;
}

extern "C" int32_t nlte_struct_size(const char* name) {
  if (!name) return -1;
  struct Entry {
    const char* n;
    size_t sz;
  };
  static const Entry tab[] = {
      {"nlte_atmos_desc", sizeof(nlte_atmos_desc)},   {"nlte_atom_desc", sizeof(nlte_atom_desc)},
      {"nlte_grid_desc", sizeof(nlte_grid_desc)},     {"nlte_solve_opts", sizeof(nlte_solve_opts)},
      {"nlte_solve_stats", sizeof(nlte_solve_stats)}, {"nlte_profile", sizeof(nlte_profile)},
      {"nlte_plan_info", sizeof(nlte_plan_info)},     {"nlte_server_result", sizeof(nlte_server_result)},
      {"nlte_server_info", sizeof(nlte_server_info)},
  };
  for (const Entry& e : tab)
    if (strcmp(e.n, name) == 0) return (int32_t)e.sz;
  return -1;
}

extern "C" nlte_status nlte_voigt_host(double a, const double* v, int32_t n, double* out) {
  if (!v || !out || n < 0) return set_err(NLTE_E_INVALID, "NULL argument");
  for (int i = 0; i < n; ++i) out[i] = voigt_H(a, v[i]);
  return NLTE_OK;
}
