// Internal layout of a column on the device and helpers shared by the
// library's HIP translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nlte.h"

namespace nlte {

// CODATA 2018, CGS.
constexpr double kH = 6.62607015e-27;
constexpr double kC = 2.99792458e10;
constexpr double kK = 1.380649e-16;
constexpr double kMe = 9.1093837015e-28;
constexpr double kAmu = 1.66053906660e-24;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;

constexpr int kWave = 64;       // lanes per wavefront (CDNA)
constexpr int kMaxMu = 8;       // angles per hemisphere held in registers
constexpr int kMaxLev = 16;     // levels per atom
constexpr int kMaxRestart = 64; // GMRES restart length

// Evaluation modes of one residual call.
enum EvalMode : int {
  kModeIdle = 0,    // column takes no part in this step
  kModeF = 1,       // F only, conservation rows taken from rows_frozen
  kModeNewton = 2,  // F, preconditioner, J; rows = most populated level
};

// One transition, packed so a wave fetches it with a few scalar loads.
struct TrDev {
  int lo, up;       // levels
  int wlo, whi;     // window on the union grid [wlo, whi)
  int voff;         // offset of its V table (lines: [nz][wlen]; edges: [wlen])
  int cwoff;        // offset of its rate weights 4 pi w / (h nu) [wlen]
  int slot;         // first partial-sum slot (one per 64-frequency chunk)
  int c0;           // first chunk it touches
  double g;         // lines: g_l / g_u
  double Blu;       // lines: Einstein B_lu (for the profile-averaged intensity)
};

// Small per-column state shared by the residual kernels and the solver.
struct ColState {
  int mode;         // EvalMode of the pending evaluation
  int want_J;       // write J of the evaluation to Jeval
  int rows_own;     // kModeF: 1 = rows from the evaluated n, 0 = rows_frozen
  int pad_rows;
  int phase;        // solver phase (see nlte_solver.hip)
  int status;       // nlte_status of the solve
  int newton_it, krylov_j, krylov_total, f_calls, stalls, ls_try, restarts, precond_calls;
  double rho_eval;  // max scaled residual of the last evaluation
  double rho_cur;   // max scaled residual at the Newton iterate
  double beta0;     // preconditioned residual norm at the start of the Newton step
  double eps_fd;    // difference step of the pending product
  double alpha;     // line-search factor
  double dn_inf;    // last population change norm
  double phi0;      // ||D^-1 P^-1 F|| at the iterate (line-search reference)
  double ftol, rtol, eps_mach, eps_scale;
  int maxiter, max_krylov, restart, max_halvings;
  int init_kind, done_flag, pad1, pad2;
};

struct ColDev {
  int nz, L, ntr, nline, nbf, nnu, nmu, prec;
  int nchunk, nslot, has_sca, N;   // N = nz * L
  // angles (inline: at most kMaxMu)
  double wm2[kMaxMu];     // w_m / 2
  double inv2mu[kMaxMu];  // 1 / (2 mu_m)
  // atmosphere
  const double *z, *dz, *T, *ne, *ntot, *chi_c, *chi_sca;
  // frequency grid and per-(k, f) tables [nz][nnu]
  const double *nu, *gam;          // gam = 2 h nu^3 / c^2
  const double *Bnu, *Ebf;         // Planck function, exp(-h nu / kT)
  // transitions
  const TrDev *tr;
  const double *V;                 // per-transition V tables
  const double *cw;                // per-transition rate weights
  const double *rho_bf;            // [nz][nbf] n*_l / n*_c
  const double *Rsp;               // [nz][ntr] n-independent part of R_ul
  const double *C_lu, *C_ul;       // [nz][ntr]
  const double *nstar;             // [nz][L]
  // chunk -> transition lists
  const int *ch_ptr, *ch_tr, *ch_slot;
  // evaluation buffers
  ColState *st;
  double *eval_n;                  // [nz][L] populations to evaluate F at
  double *F, *G;                   // [nz][L] residual and gross rates
  double *Jdag;                    // [nz][nnu] lagged mean intensity
  double *Jeval;                   // [nz][nnu] J of the last Newton-mode evaluation
  double *Jm;                      // [nz][nnu] scratch: ingoing-ray part of J
  double *Dchi, *Deta;             // [nz][nnu] scratch: ingoing-ray intensity derivatives
  double *part;                    // [nslot][nz][2] partial rate sums
  double *Ppart;                   // [nchunk][nz][L*L] partial radiative blocks
  double *P;                       // [nz][L][L] preconditioner blocks of the last Newton-mode evaluation
  double *LU;                      // [nz][L][L] LU factors of the iterate's blocks
  double *Fsave, *Gsave;           // [nz] rate-row F and gross rate under each conservation row
  double *Psave;                   // [nz][L] preconditioner row under each conservation row
  double *R;                       // [nz][ntr][2] radiative rates of the last evaluation
  double *rho_k;                   // [nz] max scaled residual per depth
  int *rows;                       // [nz] conservation rows used by the last evaluation
  int *rows_frozen;                // [nz] rows for kModeF evaluations
  int *piv;                        // [nz][L] pivots of the LU factors
  // solver buffers
  double *n;                       // [N] Newton iterate
  double *Fn;                      // [N] residual at n
  double *Vk;                      // [(m+1) N] Krylov basis
  double *H;                       // [(m+1) m] Hessenberg matrix
  double *cs, *sn, *gv;            // Givens data, [m+1]
  double *xk;                      // [N] Krylov solution (scaled unknowns)
  double *w;                       // [N] work vector
  double *lam;                     // [nz] positivity factors
  double *dots;                    // [m+1] work for orthogonalisation
};

// Formal-solution work unit: one 64-frequency chunk of one column.
struct Tile {
  int col;
  int chunk;
};

inline __host__ __device__ int chunk_of(int f) { return f / kWave; }

// Residual launches for a batch of columns (formal solution in both modes and
// precisions, then assembly).  ev, if not NULL, holds four events recorded
// before the residual-mode formal launches, after them, after the
// preconditioner-mode launches and after assembly.
hipError_t launch_residual(const ColDev* cols_dev, int ncol, const Tile* tiles_dev, int ntiles,
                           int any_fp64, int any_fp32, int any_newton, int maxL, hipStream_t s,
                           hipEvent_t* ev = nullptr);

}  // namespace nlte

struct nlte_ctx {
  int device;
  int prof_on;
  nlte_profile prof;
};
