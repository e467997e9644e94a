// Jacobian-free Newton-Krylov solve (Algorithm 2) on the device.
//
// Every column carries its own Newton/Krylov state in device memory.  A solve
// advances in steps; in each step every active column evaluates exactly one
// residual (the pending evaluation set up by the previous step) and then one
// block per column consumes it:
//   INIT      F(n0) with preconditioner            -> start GMRES
//   ARNOLDI   F(n + eps D v_j) (frozen rows)        -> one Arnoldi step
//   RESTART   F(n + eps D x)                        -> restarted residual
//   LINESRCH  F(n + alpha lambda D u) with P and J  -> accept or halve alpha
// so the host only replays the same launches until every column is done.
// The Krylov unknowns are relative corrections u = D^-1 dn with D = diag(n)
// (Sect. 2.4.2 notes the rescaling); the system is left-preconditioned with
// the block-Jacobi P (Eq. prec2), GMRES(m) uses classical Gram-Schmidt with
// one re-orthogonalisation, and Newton steps are limited per depth to keep
// populations positive and damped by backtracking (Sect. 2.2.2).
#include <math.h>

#include <vector>

#include "nlte_internal.h"

nlte_status set_err(nlte_status st, const char* fmt, ...);

namespace nlte {
const ColDev& column_dev(const nlte_column* c);
ColDev* column_dev_ptr(const nlte_column* c);
int column_restart_cap(const nlte_column* c);
nlte_ctx* column_ctx(const nlte_column* c);
void transpose_J(const ColDev& C, double* out, hipStream_t s);
}  // namespace nlte

using namespace nlte;

namespace {

constexpr int kThreads = 256;
constexpr int kMaxM = 32;  // restart capacity allocated per column
// Noise level assumed for the forward-difference step of FP32-form columns.
// After the cancellations between gross rates, the FP32 formal solution
// leaves relative noise far above 2^-23 in F; steps built on the FP32 machine
// epsilon drown Jv in it.  Noise levels 1e-4..1e-2 all give converging
// Newton sequences on the 6-level chromosphere; 1e-3 sits in the middle.
constexpr double kFp32Noise = 1e-3;
constexpr double kEpsMach64 = 2.220446049250313e-16;
// An FP32-form column that falls back to FP64 keeps its iterate when its
// max |F|/gross-rate is at most this (on the 6-level batch these are mostly
// columns stalled at the FP32 noise floor just above the tolerance, which
// FP64 finishes in one or two Newton iterations); one further from the root
// starts again from its initial populations.
constexpr double kFallbackKeepRho = 1e-2;

enum Phase : int {
  PH_IDLE = 0, PH_INIT = 1, PH_ARNOLDI = 2, PH_RESTART = 3, PH_LS = 4, PH_DONE = 5,
  PH_BICG_V = 6,  // BiCGSTAB: the product A p is pending
  PH_BICG_T = 7,  // BiCGSTAB: the product A s is pending
  PH_X0 = 8       // the product A x0 of a nonzero initial guess is pending
};

// ----------------------------------------------------------------- block ops
__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double warp_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o));
  return v;
}

// Sums `cnt` per-thread partials (cnt <= kMaxM + 1) over the block; result in out[0..cnt).
__device__ void block_sums(double* part, int cnt, double* red, double* out) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = 0; i < cnt; ++i) {
    const double s = warp_sum(part[i]);
    if (lane == 0) red[wave * (kMaxM + 1) + i] = s;
  }
  __syncthreads();
  if (tid < cnt) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w * (kMaxM + 1) + tid];
    out[tid] = s;
  }
  __syncthreads();
}

__device__ double block_sum1(double v, double* red) {
  double p[1] = {v};
  __shared__ double o[1];
  block_sums(p, 1, red, o);
  return o[0];
}

__device__ double block_max1(double v, double* red) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double m = warp_max(v);
  if (lane == 0) red[wave] = m;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < kThreads / 64; ++w) r = nanmax(r, red[w]);
  __syncthreads();
  return r;
}

// ------------------------------------------------------- per-depth dense LU
// In-place LU with partial pivoting of a row-major L x L block.
__device__ bool lu_factor(double* A, int* piv, int L) {
  bool ok = true;
  for (int c = 0; c < L; ++c) {
    int p = c;
    double best = fabs(A[c * L + c]);
    for (int r = c + 1; r < L; ++r) {
      const double v = fabs(A[r * L + c]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    piv[c] = p;
    if (p != c)
      for (int j = 0; j < L; ++j) {
        const double t = A[c * L + j];
        A[c * L + j] = A[p * L + j];
        A[p * L + j] = t;
      }
    const double d = A[c * L + c];
    if (d == 0.0 || d != d) {
      ok = false;
      continue;
    }
    const double inv = 1.0 / d;
    for (int r = c + 1; r < L; ++r) {
      const double f = A[r * L + c] * inv;
      A[r * L + c] = f;
      for (int j = c + 1; j < L; ++j) A[r * L + j] -= f * A[c * L + j];
    }
  }
  return ok;
}

__device__ void lu_solve(const double* A, const int* piv, double* x, int L) {
  for (int c = 0; c < L; ++c) {
    const int p = piv[c];
    if (p != c) {
      const double t = x[c];
      x[c] = x[p];
      x[p] = t;
    }
  }
  for (int r = 1; r < L; ++r) {
    double s = x[r];
    for (int c = 0; c < r; ++c) s -= A[r * L + c] * x[c];
    x[r] = s;
  }
  for (int r = L - 1; r >= 0; --r) {
    double s = x[r];
    for (int c = r + 1; c < L; ++c) s -= A[r * L + c] * x[c];
    x[r] = s / A[r * L + r];
  }
}

// The LU solve with the level count fixed at compile time, so that the
// right-hand side stays in registers (atoms of up to 8 levels; larger blocks
// take the general loop below, whose vector lives in private memory; fixing
// those too raised the solver kernel's register count for every column).
template <int L>
__device__ __forceinline__ void pinv_depths(const ColDev& C, const double* in, double* out) {
  for (int k = threadIdx.x; k < C.nz; k += kThreads) {
    const double* A = C.LU + (size_t)k * L * L;
    const int* piv = C.piv + k * L;
    double x[L];
#pragma unroll
    for (int i = 0; i < L; ++i) x[i] = in[k * L + i];
#pragma unroll
    for (int c = 0; c < L; ++c) {
      const int p = piv[c];
      // swap x[c] and x[p] (p >= c) without a runtime register index
      double xp = x[c];
#pragma unroll
      for (int r = c + 1; r < L; ++r)
        if (r == p) xp = x[r];
#pragma unroll
      for (int r = c + 1; r < L; ++r)
        if (r == p) x[r] = x[c];
      x[c] = xp;
    }
#pragma unroll
    for (int r = 1; r < L; ++r) {
      double t = x[r];
#pragma unroll
      for (int c = 0; c < r; ++c) t -= A[r * L + c] * x[c];
      x[r] = t;
    }
#pragma unroll
    for (int r = L - 1; r >= 0; --r) {
      double t = x[r];
#pragma unroll
      for (int c = r + 1; c < L; ++c) t -= A[r * L + c] * x[c];
      x[r] = t / A[r * L + r];
    }
#pragma unroll
    for (int i = 0; i < L; ++i) out[k * L + i] = x[i] / C.n[k * L + i];
  }
}

__device__ void pinv_depths_any(const ColDev& C, const double* in, double* out) {
  const int L = C.L;
  for (int k = threadIdx.x; k < C.nz; k += kThreads) {
    double x[kMaxLev];
    for (int i = 0; i < L; ++i) x[i] = in[k * L + i];
    lu_solve(C.LU + (size_t)k * L * L, C.piv + k * L, x, L);
    for (int i = 0; i < L; ++i) out[k * L + i] = x[i] / C.n[k * L + i];
  }
}

// out = D^-1 P^-1 in (per depth), in/out may alias; D = diag(n).
__device__ void apply_scaled_pinv(const ColDev& C, const double* in, double* out) {
  switch (C.L) {
    case 2: pinv_depths<2>(C, in, out); break;
    case 3: pinv_depths<3>(C, in, out); break;
    case 4: pinv_depths<4>(C, in, out); break;
    case 5: pinv_depths<5>(C, in, out); break;
    case 6: pinv_depths<6>(C, in, out); break;
    case 7: pinv_depths<7>(C, in, out); break;
    case 8: pinv_depths<8>(C, in, out); break;
    default: pinv_depths_any(C, in, out); break;
  }
  __syncthreads();
}

__device__ void finish(const ColDev& C, int status, int* done_count) {
  if (threadIdx.x == 0) {
    C.st->status = status;
    C.st->phase = PH_DONE;
    C.st->mode = kModeIdle;
    atomicAdd(done_count, 1);
  }
}

// The product J D v of the next step.  Forward difference (Eq. fordif):
// eval_n = n (1 + eps v), the perturbed state.  Tangent (Eq. complex in the
// limit of a vanishing step): eval_n = D v = n v, the direction, with the
// column's residual kernels idle and its tangent kernels on.
__device__ void prepare_jv(const ColDev& C, const double* v, double vnorm) {
  ColState* st = C.st;
  if (st->jv == NLTE_JV_TANGENT) {
    for (int i = threadIdx.x; i < C.N; i += kThreads) C.eval_n[i] = C.n[i] * v[i];
    if (threadIdx.x == 0) {
      st->mode = kModeIdle;
      st->tan_pending = 1;
      st->want_J = 0;
    }
    return;
  }
  const double eps = st->eps_scale * sqrt(st->eps_mach) * sqrt(1.0 + sqrt((double)C.N)) / vnorm;
  for (int i = threadIdx.x; i < C.N; i += kThreads) C.eval_n[i] = C.n[i] * (1.0 + eps * v[i]);
  if (threadIdx.x == 0) {
    st->eps_fd = eps;
    st->mode = kModeF;
    st->rows_own = 0;
    st->want_J = 0;
  }
}

// r in Vk[0] (unnormalised): start a GMRES cycle
__device__ void start_cycle(const ColDev& C, bool first, double* red, int* done_count) {
  ColState* st = C.st;
  double p = 0.0;
  for (int i = threadIdx.x; i < C.N; i += kThreads) p += C.Vk[i] * C.Vk[i];
  const double beta = sqrt(block_sum1(p, red));
  if (first && threadIdx.x == 0) {
    st->beta0 = beta;
    st->phi0 = beta;
  }
  if (!(beta > 0.0) || beta != beta) {
    // F vanishes in the preconditioned norm: nothing left to correct
    if (beta != beta) finish(C, NLTE_E_NONFINITE, done_count);
    else finish(C, NLTE_OK, done_count);
    return;
  }
  const double ib = 1.0 / beta;
  for (int i = threadIdx.x; i < C.N; i += kThreads) C.Vk[i] *= ib;
  if (threadIdx.x == 0) {
    C.gv[0] = beta;
    for (int i = 1; i <= kMaxM; ++i) C.gv[i] = 0.0;
    for (int i = 0; i < (kMaxM + 1) * kMaxM; ++i) C.H[i] = 0.0;
    st->krylov_j = 0;
    st->phase = PH_ARNOLDI;
  }
  __syncthreads();
  prepare_jv(C, C.Vk, 1.0);
}

__device__ void begin_linesearch(const ColDev& C) {
  ColState* st = C.st;
  const int L = C.L;
  // per-depth limit (Sect. 2.2.2): with u = dn / n, every level of
  // n (1 + lambda u) stays within [n / 3, 3 n]
  for (int k = threadIdx.x; k < C.nz; k += kThreads) {
    double dec = 0.0, inc = 0.0;
    for (int i = 0; i < L; ++i) {
      dec = fmax(dec, -C.xk[k * L + i]);
      inc = fmax(inc, C.xk[k * L + i]);
    }
    double lam = 1.0;
    if (dec > 0.0) lam = fmin(lam, (2.0 / 3.0) / dec);
    if (inc > 0.0) lam = fmin(lam, 2.0 / inc);
    C.lam[k] = lam;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < C.N; i += kThreads)
    C.eval_n[i] = C.n[i] * (1.0 + C.lam[i / L] * C.xk[i]);
  if (threadIdx.x == 0) {
    st->alpha = 1.0;
    st->ls_try = 0;
    st->phase = PH_LS;
    st->mode = kModeNewton;
    st->rows_own = 0;
    st->want_J = 1;
  }
}

// ---------------------------------------------------------------------------
// BiCGSTAB (Sect. 2.3, the paper's second inner solver) on the same
// left-preconditioned, scaled system A x = b as GMRES, A = D^-1 P^-1 J D,
// b = -D^-1 P^-1 F(n), x0 = 0, shadow residual r^ = b.  Each product A u is
// one residual evaluation at n (1 + eps u), so an iteration spans two steps
// of the state machine.  Vectors in the Krylov slots: 0 r^, 1 r, 2 p,
// 3 v = A p, 4 s, 5 t = A s; x in xk.
// ---------------------------------------------------------------------------
// Whether the product just made exhausts the Krylov budget, from the counters
// as they were before it (read by every thread before thread 0 advances them,
// so that the whole block takes the same branch).
__device__ __forceinline__ bool krylov_capped_after(const ColState* st, int ks, int kt) {
  return ks + 1 >= st->max_krylov || (st->max_krylov_total > 0 && kt + 1 >= st->max_krylov_total);
}

// J D v of the evaluation just made: (F - F(n)) / eps for a forward
// difference, F itself for a tangent product
__device__ void product_into(const ColDev& C, double* w) {
  if (C.st->jv == NLTE_JV_TANGENT) {
    for (int i = threadIdx.x; i < C.N; i += kThreads) w[i] = C.F[i];
  } else {
    const double ieps = 1.0 / C.st->eps_fd;
    for (int i = threadIdx.x; i < C.N; i += kThreads) w[i] = (C.F[i] - C.Fn[i]) * ieps;
  }
  __syncthreads();
}

// w = D^-1 P^-1 J D v: the product of the pending evaluation
__device__ void pending_product(const ColDev& C, double* w) {
  product_into(C, w);
  apply_scaled_pinv(C, w, w);
}

// first: the Krylov solve starts here from x0 = 0, so ||r0|| = ||b|| is the
// reference of its tolerance and of the line search; otherwise (nonzero x0)
// that reference was set when b was formed.
__device__ void bicg_start(const ColDev& C, bool first, double* red, int* done_count) {
  ColState* st = C.st;
  const int N = C.N;
  double* rh = C.Vk;
  double* r = C.Vk + N;
  double* p = C.Vk + 2 * (size_t)N;
  double q = 0.0;
  for (int i = threadIdx.x; i < N; i += kThreads) {
    const double b = rh[i];
    r[i] = b;
    p[i] = b;
    q += b * b;
  }
  const double bb = block_sum1(q, red);
  const double beta = sqrt(bb);
  if (!(beta > 0.0) || beta != beta) {
    // F vanishes in the preconditioned norm: nothing left to correct
    if (beta != beta) finish(C, NLTE_E_NONFINITE, done_count);
    else finish(C, NLTE_OK, done_count);
    return;
  }
  if (threadIdx.x == 0) {
    if (first) {
      st->beta0 = beta;
      st->phi0 = beta;
    }
    st->bi_rho = bb;  // (r^, r0) with r^ = r0
    st->phase = PH_BICG_V;
  }
  prepare_jv(C, p, beta);
}

// A p has been evaluated: alpha, s = r - alpha v; stop on s, else evaluate A s
__device__ void bicg_v(const ColDev& C, double* red, int* done_count) {
  ColState* st = C.st;
  const int N = C.N;
  const double rho = st->bi_rho, rtol = st->rtol, beta0 = st->beta0;
  const bool capped = krylov_capped_after(st, st->krylov_step, st->krylov_total);
  double* rh = C.Vk;
  double* r = C.Vk + N;
  double* p = C.Vk + 2 * (size_t)N;
  double* v = C.Vk + 3 * (size_t)N;
  double* sv = C.Vk + 4 * (size_t)N;
  pending_product(C, v);
  double q = 0.0;
  for (int i = threadIdx.x; i < N; i += kThreads) q += rh[i] * v[i];
  const double den = block_sum1(q, red);
  __syncthreads();  // every thread has read the state before thread 0 changes it
  if (threadIdx.x == 0) {
    st->krylov_total += 1;
    st->krylov_step += 1;
  }
  const double alpha = rho / den;
  if (!(den != 0.0) || !isfinite(alpha)) {  // breakdown: keep x as it is
    begin_linesearch(C);
    return;
  }
  double ss = 0.0;
  for (int i = threadIdx.x; i < N; i += kThreads) {
    const double si = r[i] - alpha * v[i];
    sv[i] = si;
    ss += si * si;
  }
  const double sn = sqrt(block_sum1(ss, red));
  if (sn <= rtol * beta0 || capped) {
    for (int i = threadIdx.x; i < N; i += kThreads) C.xk[i] += alpha * p[i];
    __syncthreads();
    begin_linesearch(C);
    return;
  }
  if (threadIdx.x == 0) {
    st->bi_alpha = alpha;
    st->phase = PH_BICG_T;
  }
  prepare_jv(C, sv, sn);
}

// A s has been evaluated: omega, x += alpha p + omega s, r = s - omega t;
// stop on r, else the next direction p and its product
__device__ void bicg_t(const ColDev& C, double* red, int* done_count) {
  ColState* st = C.st;
  const int N = C.N;
  const double rho = st->bi_rho, alpha = st->bi_alpha, rtol = st->rtol, beta0 = st->beta0;
  const bool capped = krylov_capped_after(st, st->krylov_step, st->krylov_total);
  double* rh = C.Vk;
  double* r = C.Vk + N;
  double* p = C.Vk + 2 * (size_t)N;
  double* v = C.Vk + 3 * (size_t)N;
  double* sv = C.Vk + 4 * (size_t)N;
  double* t = C.Vk + 5 * (size_t)N;
  pending_product(C, t);
  __shared__ double d2[2];
  double part[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < N; i += kThreads) {
    part[0] += t[i] * t[i];
    part[1] += t[i] * sv[i];
  }
  block_sums(part, 2, red, d2);
  const double tt = d2[0], ts = d2[1];
  const double omega = tt > 0.0 ? ts / tt : 0.0;
  double part2[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < N; i += kThreads) {
    C.xk[i] += alpha * p[i] + omega * sv[i];
    const double ri = sv[i] - omega * t[i];
    r[i] = ri;
    part2[0] += ri * ri;
    part2[1] += rh[i] * ri;
  }
  __shared__ double e2[2];
  block_sums(part2, 2, red, e2);
  const double rn = sqrt(e2[0]), rho_new = e2[1];
  __syncthreads();  // every thread has read the state before thread 0 changes it
  if (threadIdx.x == 0) {
    st->krylov_total += 1;
    st->krylov_step += 1;
  }
  const double beta = (rho_new / rho) * (alpha / omega);
  if (rn <= rtol * beta0 || capped || !(omega != 0.0) || !(rho_new != 0.0) ||
      !isfinite(beta)) {
    __syncthreads();
    begin_linesearch(C);
    return;
  }
  double pp = 0.0;
  for (int i = threadIdx.x; i < N; i += kThreads) {
    const double pi = r[i] + beta * (p[i] - omega * v[i]);
    p[i] = pi;
    pp += pi * pi;
  }
  const double pn = sqrt(block_sum1(pp, red));
  if (threadIdx.x == 0) {
    st->bi_rho = rho_new;
    st->phase = PH_BICG_V;
  }
  prepare_jv(C, p, pn);
}

// The pending evaluation was a Newton-mode F at eval_n: make it the iterate.
// Its conservation rows move to the most populated levels of eval_n (the
// rate rows they replace were saved by the assembly, so this needs no new
// formal solution), then the preconditioner blocks are factored and a GMRES
// cycle starts on b = -D^-1 P^-1 F.
//
// Lagged scattering (Sect. 2.1.1, Algorithm 2 "update J"): at a newly
// accepted point of a column with background scattering, J-dagger first
// becomes the J of the evaluation just made, and F is evaluated again at the
// same point with it; the Newton step then starts from that second
// evaluation, so that F(n), its products and its line search share one
// J-dagger (the difference of Eq. fordif would otherwise pick up the change
// of J-dagger between its two terms).  The first evaluation of a solve (and
// of an FP64 fallback) keeps the J-dagger it was given.
__device__ void accept_point(const ColDev& C, double* red, int* done_count) {
  ColState* st = C.st;
  const int N = C.N, L = C.L;
  const bool refresh = C.has_sca && !st->jdag_fresh;
  __syncthreads();  // every thread has read the state before thread 0 changes it
  if (refresh) {
    for (int i = threadIdx.x; i < C.nz * C.nnu; i += kThreads) {
      const int k = i / C.nnu, f = i - k * C.nnu;
      C.Jdag[i] = C.JT[(size_t)f * C.zp + k];
    }
    if (threadIdx.x == 0) {
      st->jdag_fresh = 1;
      st->phase = PH_INIT;
      st->mode = kModeNewton;
      st->rows_own = 1;
      st->want_J = 1;
    }
    return;
  }
  if (threadIdx.x == 0) st->jdag_fresh = 0;
  double rk = 0.0;
  for (int k = threadIdx.x; k < C.nz; k += kThreads) {
    const double* nk = C.eval_n + k * L;
    int rn = 0;
    for (int i = 1; i < L; ++i)
      if (nk[i] > nk[rn]) rn = i;
    const int ro = C.rows[k];
    if (rn != ro) {
      double sum = 0.0;
      for (int i = 0; i < L; ++i) sum += nk[i];
      C.F[k * L + ro] = C.Fsave[k];
      C.G[k * L + ro] = C.Gsave[k];
      C.Fsave[k] = C.F[k * L + rn];
      C.Gsave[k] = C.G[k * L + rn];
      C.F[k * L + rn] = C.ntot[k] - sum;
      C.G[k * L + rn] = C.ntot[k];
      double* Pk = C.P + (size_t)k * L * L;
      for (int j = 0; j < L; ++j) {
        Pk[ro * L + j] = C.Psave[k * L + j];
        C.Psave[k * L + j] = Pk[rn * L + j];
        Pk[rn * L + j] = -1.0;
      }
    }
    C.rows_frozen[k] = rn;
    for (int i = 0; i < L; ++i) {
      const double q = fabs(C.F[k * L + i]) / C.G[k * L + i];
      rk = nanmax(rk, q);
    }
  }
  const double rho = block_max1(rk, red);
  for (int i = threadIdx.x; i < N; i += kThreads) {
    C.n[i] = C.eval_n[i];
    C.Fn[i] = C.F[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) st->rho_cur = rho;
  if (rho != rho || isinf(rho)) {
    finish(C, NLTE_E_NONFINITE, done_count);
    return;
  }
  if (rho <= st->ftol) {
    finish(C, NLTE_OK, done_count);
    return;
  }
  const bool fallback = st->cur_prec == NLTE_FP32_FORM && st->fp64_fallback > 0 &&
                        st->newton_it >= st->fp64_fallback && st->newton_it < st->maxiter;
  __syncthreads();  // every thread has read the state before thread 0 changes it
  if (fallback) {
    // FP32 form not converging: continue with FP64 formal solutions (own
    // rows, new P), from the current iterate when it is close to the root,
    // else from the initial populations (an iterate the FP32 Newton sequence
    // wandered to is often a poor start).  eval_n and Jdag hold the current
    // iterate and its J.
    if (!(rho <= kFallbackKeepRho)) {
      for (int i = threadIdx.x; i < C.N; i += kThreads) C.eval_n[i] = C.n_init[i];
      if (C.has_sca)
        for (int i = threadIdx.x; i < C.nz * C.nnu; i += kThreads) C.Jdag[i] = C.Bnu[i];
    }
    if (threadIdx.x == 0) {
      st->jdag_fresh = 1;  // the fallback's first evaluation keeps its J-dagger
      st->cur_prec = NLTE_FP64;
      st->eps_mach = kEpsMach64;
      st->krylov_total = 0;
      st->phase = PH_INIT;
      st->mode = kModeNewton;
      st->rows_own = 1;
      st->want_J = 1;
    }
    return;
  }
  if (st->newton_it >= st->maxiter) {
    finish(C, NLTE_E_NOCONV, done_count);
    return;
  }
  // factor the preconditioner blocks into LU
  int bad = 0;
  for (int k = threadIdx.x; k < C.nz; k += kThreads) {
    double* A = C.LU + (size_t)k * L * L;
    const double* Pk = C.P + (size_t)k * L * L;
    for (int q = 0; q < L * L; ++q) A[q] = Pk[q];
    if (!lu_factor(A, C.piv + k * L, L)) bad = 1;
  }
  const double anybad = block_max1((double)bad, red);
  if (anybad > 0.0) {
    finish(C, NLTE_E_NONFINITE, done_count);
    return;
  }
  // b = -D^-1 P^-1 F(n) -> Vk[0]
  apply_scaled_pinv(C, C.Fn, C.Vk);
  const bool x0 = st->krylov_x0 != 0;
  double bb = 0.0;
  for (int i = threadIdx.x; i < N; i += kThreads) {
    const double b = -C.Vk[i];
    C.Vk[i] = b;
    C.xk[i] = x0 ? b : 0.0;  // x0 = -P^-1 F in the unscaled unknowns is b here
    bb += b * b;
  }
  if (threadIdx.x == 0) {
    st->restarts = 0;
    st->krylov_step = 0;
  }
  if (x0) {
    // the Krylov solve starts from r0 = b - A x0: evaluate A x0 first
    const double bn = sqrt(block_sum1(bb, red));
    if (!(bn > 0.0) || bn != bn) {
      if (bn != bn) finish(C, NLTE_E_NONFINITE, done_count);
      else finish(C, NLTE_OK, done_count);
      return;
    }
    if (threadIdx.x == 0) {
      st->beta0 = bn;
      st->phi0 = bn;
      st->phase = PH_X0;
    }
    prepare_jv(C, C.xk, bn);
    return;
  }
  __syncthreads();
  if (st->method == NLTE_KRYLOV_BICGSTAB)
    bicg_start(C, true, red, done_count);
  else
    start_cycle(C, true, red, done_count);
}

// A x0 has been evaluated: r0 = b - A x0 replaces b in Vk[0] and the Krylov
// solve starts from x = x0 (its tolerance and the line search still refer to
// ||b||, set when b was formed).
__device__ void x0_product(const ColDev& C, double* red, int* done_count) {
  ColState* st = C.st;
  double* w = C.w;
  pending_product(C, w);
  for (int i = threadIdx.x; i < C.N; i += kThreads) C.Vk[i] -= w[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    st->krylov_total += 1;
    st->krylov_step += 1;
  }
  __syncthreads();
  if (st->method == NLTE_KRYLOV_BICGSTAB)
    bicg_start(C, false, red, done_count);
  else
    start_cycle(C, false, red, done_count);
}

__device__ void arnoldi(const ColDev& C, double* red, int* done_count) {
  ColState* st = C.st;
  const int N = C.N, m = st->restart;
  const int j = st->krylov_j;
  double* w = C.w;
  product_into(C, w);
  apply_scaled_pinv(C, w, w);
  // classical Gram-Schmidt, twice; the j + 1 dot products go to the waves
  // four basis vectors at a time (lane-strided sums, then a wave reduction)
  __shared__ double h[kMaxM + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int pass = 0; pass < 2; ++pass) {
    for (int i0 = 4 * wave; i0 <= j; i0 += 4 * (kThreads / 64)) {
      const int ni = min(4, j + 1 - i0);
      const double* v0 = C.Vk + (size_t)i0 * N;
      double d[4] = {0.0, 0.0, 0.0, 0.0};
      for (int q = lane; q < N; q += 64) {
        const double wq = w[q];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (u < ni) d[u] = fma(v0[(size_t)u * N + q], wq, d[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double t = warp_sum(d[u]);
        if (lane == 0 && u < ni) h[i0 + u] = t;
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < N; q += kThreads) {
      double s = w[q];
      for (int i = 0; i <= j; ++i) s -= h[i] * C.Vk[(size_t)i * N + q];
      w[q] = s;
    }
    if (threadIdx.x <= j) C.H[threadIdx.x * kMaxM + j] += h[threadIdx.x];
    __syncthreads();
  }
  double p = 0.0;
  for (int q = threadIdx.x; q < N; q += kThreads) p += w[q] * w[q];
  const double hn = sqrt(block_sum1(p, red));
  const bool brk = !(hn > 1e-300);
  if (!brk) {
    const double ih = 1.0 / hn;
    for (int q = threadIdx.x; q < N; q += kThreads) C.Vk[(size_t)(j + 1) * N + q] = w[q] * ih;
  }
  __shared__ double s_resid;
  if (threadIdx.x == 0) {
    double* H = C.H;
    H[(j + 1) * kMaxM + j] = hn;
    for (int i = 0; i < j; ++i) {
      const double a = H[i * kMaxM + j], b = H[(i + 1) * kMaxM + j];
      H[i * kMaxM + j] = C.cs[i] * a + C.sn[i] * b;
      H[(i + 1) * kMaxM + j] = -C.sn[i] * a + C.cs[i] * b;
    }
    const double a = H[j * kMaxM + j], b = H[(j + 1) * kMaxM + j];
    const double den = hypot(a, b);
    C.cs[j] = den > 0 ? a / den : 1.0;
    C.sn[j] = den > 0 ? b / den : 0.0;
    H[j * kMaxM + j] = den;
    H[(j + 1) * kMaxM + j] = 0.0;
    C.gv[j + 1] = -C.sn[j] * C.gv[j];
    C.gv[j] = C.cs[j] * C.gv[j];
    s_resid = fabs(C.gv[j + 1]);
    st->krylov_j = j + 1;
    st->krylov_total += 1;
    st->krylov_step += 1;
  }
  __syncthreads();
  const int jj = j + 1;
  const bool conv = s_resid <= st->rtol * st->beta0;
  const bool cap = st->krylov_step >= st->max_krylov ||  // per Newton step
                   (st->max_krylov_total > 0 && st->krylov_total >= st->max_krylov_total);
  if (!(conv || cap || brk || jj == m)) {
    prepare_jv(C, C.Vk + (size_t)jj * N, 1.0);
    return;
  }
  // y = H^-1 g (upper triangular jj x jj), x += V y
  __shared__ double y[kMaxM];
  if (threadIdx.x == 0) {
    for (int r = jj - 1; r >= 0; --r) {
      double s = C.gv[r];
      for (int c = r + 1; c < jj; ++c) s -= C.H[r * kMaxM + c] * y[c];
      const double d = C.H[r * kMaxM + r];
      y[r] = d != 0.0 ? s / d : 0.0;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < N; q += kThreads) {
    double s = C.xk[q];
    for (int i = 0; i < jj; ++i) s += y[i] * C.Vk[(size_t)i * N + q];
    C.xk[q] = s;
  }
  __syncthreads();
  if (conv || cap || brk) {
    begin_linesearch(C);
    return;
  }
  // restart: evaluate A x for the true residual b - A x
  double px = 0.0;
  for (int q = threadIdx.x; q < N; q += kThreads) px += C.xk[q] * C.xk[q];
  const double xn = sqrt(block_sum1(px, red));
  if (threadIdx.x == 0) {
    st->phase = PH_RESTART;
    st->restarts += 1;
  }
  if (!(xn > 0.0)) {
    begin_linesearch(C);
    return;
  }
  prepare_jv(C, C.xk, xn);
}

__device__ void restart(const ColDev& C, double* red, int* done_count) {
  const int N = C.N;
  double* w = C.w;
  product_into(C, w);
  apply_scaled_pinv(C, w, w);           // A x
  apply_scaled_pinv(C, C.Fn, C.Vk);     // -b
  for (int i = threadIdx.x; i < N; i += kThreads) C.Vk[i] = -C.Vk[i] - w[i];
  __syncthreads();
  start_cycle(C, false, red, done_count);
}

// Backtracking (Sect. 2.2.2) on the norm the Krylov step reduces:
// accept the trial when ||D^-1 P^-1 F(trial)||_2 < (1 - 1e-4 alpha) ||D^-1 P^-1 F(n)||_2
// with the iterate's P, D and conservation rows; else halve alpha.
__device__ void linesearch(const ColDev& C, double* red, int* done_count) {
  ColState* st = C.st;
  const int N = C.N, L = C.L;
  apply_scaled_pinv(C, C.F, C.w);
  double p = 0.0;
  for (int i = threadIdx.x; i < N; i += kThreads) p += C.w[i] * C.w[i];
  const double phi = sqrt(block_sum1(p, red));
  const double alpha = st->alpha;
  const bool ok = phi < (1.0 - 1e-4 * alpha) * st->phi0;
  if (ok || st->ls_try >= st->max_halvings) {
    if (!ok && (phi != phi || isinf(phi))) {
      finish(C, NLTE_E_NONFINITE, done_count);
      return;
    }
    double q = 0.0;
    for (int i = threadIdx.x; i < N; i += kThreads)
      q = fmax(q, fabs((C.eval_n[i] - C.n[i]) / (C.eval_n[i] + C.n[i])));
    const double dn = 0.5 * block_max1(q, red);
    if (threadIdx.x == 0) {
      st->dn_inf = dn;
      st->newton_it += 1;
      if (!ok) st->stalls += 1;
    }
    __syncthreads();
    accept_point(C, red, done_count);
    return;
  }
  const double a2 = 0.5 * alpha;
  for (int i = threadIdx.x; i < N; i += kThreads)
    C.eval_n[i] = C.n[i] * (1.0 + a2 * C.lam[i / L] * C.xk[i]);
  __syncthreads();
  if (threadIdx.x == 0) {
    st->alpha = a2;
    st->ls_try += 1;
  }
}

__global__ __launch_bounds__(kThreads) void k_solver_step(const ColDev* __restrict__ cols,
                                                          const int* __restrict__ act,
                                                          int* done_count) {
  __shared__ double red[(kThreads / 64) * (kMaxM + 1)];
  __shared__ int s_phase;
  const ColDev& C = cols[act ? act[blockIdx.x] : blockIdx.x];
  if (threadIdx.x == 0) {
    s_phase = C.st->phase;
    C.st->tan_pending = 0;  // the tangent product (if any) has been made
    if (s_phase != PH_DONE && s_phase != PH_IDLE) {
      C.st->f_calls += 1;
      if (C.prec == NLTE_FP32_FORM && C.st->cur_prec == NLTE_FP64) C.st->fp64_evals += 1;
    }
    if (s_phase == PH_INIT || s_phase == PH_LS) C.st->precond_calls += 1;
  }
  __syncthreads();
  const int phase = s_phase;
  switch (phase) {
    case PH_INIT: accept_point(C, red, done_count); break;
    case PH_ARNOLDI: arnoldi(C, red, done_count); break;
    case PH_RESTART: restart(C, red, done_count); break;
    case PH_LS: linesearch(C, red, done_count); break;
    case PH_BICG_V: bicg_v(C, red, done_count); break;
    case PH_BICG_T: bicg_t(C, red, done_count); break;
    case PH_X0: x0_product(C, red, done_count); break;
    default: break;
  }
}

// Solve setup: options, initial populations, J-dagger = B, first evaluation.
struct InitArgs {
  double ftol, rtol, eps_mach, eps_scale;
  int maxiter, max_krylov, restart, max_halvings, init, max_krylov_total, fp64_fallback, method, jv;
  int x0;
};

__global__ void k_solver_init(const ColDev* __restrict__ cols, const double* const* n0,
                              const double* const* J0, InitArgs a) {
  const ColDev& C = cols[blockIdx.x];
  ColState* st = C.st;
  const double* src = n0 ? n0[blockIdx.x] : nullptr;
  for (int i = threadIdx.x; i < C.N; i += blockDim.x) {
    const double v = (a.init == 0 && src) ? src[i] : C.nstar[i];
    C.eval_n[i] = v;
    C.n_init[i] = v;
  }
  const double* jsrc = J0 ? J0[blockIdx.x] : nullptr;
  const double* jin = jsrc ? jsrc : C.Bnu;
  for (int i = threadIdx.x; i < C.nz * C.nnu; i += blockDim.x) C.Jdag[i] = jin[i];
  if (threadIdx.x == 0) {
    st->phase = PH_INIT;
    st->status = NLTE_E_NOCONV;
    st->newton_it = 0;
    st->krylov_j = 0;
    st->krylov_total = 0;
    st->krylov_step = 0;
    st->f_calls = 0;
    st->precond_calls = 0;
    st->stalls = 0;
    st->ls_try = 0;
    st->restarts = 0;
    st->rho_cur = 0;
    st->dn_inf = 0;
    st->ftol = a.ftol;
    st->rtol = a.rtol;
    st->eps_mach = C.prec == NLTE_FP32_FORM ? kFp32Noise : a.eps_mach;
    st->eps_scale = a.eps_scale;
    st->maxiter = a.maxiter;
    st->max_krylov = a.max_krylov;
    st->max_krylov_total = a.max_krylov_total;
    st->cur_prec = C.prec;
    st->fp64_fallback = a.fp64_fallback;
    st->method = a.method;
    st->jv = a.jv;
    st->krylov_x0 = a.x0;
    st->tan_pending = 0;
    st->fp64_evals = 0;
    st->restart = a.restart;
    st->max_halvings = a.max_halvings;
    st->mode = kModeNewton;
    st->rows_own = 1;
    st->want_J = 1;
    st->jdag_fresh = 1;  // F(n0) uses the J-dagger the solve starts with
  }
}

// Radiation-free populations: per depth, rate equations with J = 0 (R_lu = 0,
// R_ul = its spontaneous part) plus particle conservation on the most
// populated level of the result (re-solved while that level changes).
__global__ void k_zero_radiation(const ColDev* __restrict__ cols, double* out) {
  const ColDev& C = cols[0];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= C.nz) return;
  const int L = C.L;
  double M0[kMaxLev * kMaxLev];
  for (int i = 0; i < L * L; ++i) M0[i] = 0.0;
  for (int t = 0; t < C.ntr; ++t) {
    const TrDev T = C.tr[t];
    const double Rul = (t < C.nline) ? T.g * C.Rsp[k * C.ntr + t]
                                     : C.rho_bf[k * C.nbf + (t - C.nline)] * C.Rsp[k * C.ntr + t];
    const double up = C.C_lu[k * C.ntr + t], dn = C.C_ul[k * C.ntr + t] + Rul;
    M0[T.lo * L + T.lo] += up;
    M0[T.up * L + T.up] += dn;
    M0[T.lo * L + T.up] -= dn;
    M0[T.up * L + T.lo] -= up;
  }
  int row = 0;
  for (int i = 1; i < L; ++i)
    if (C.nstar[k * L + i] > C.nstar[k * L + row]) row = i;
  double A[kMaxLev * kMaxLev], x[kMaxLev];
  int piv[kMaxLev];
  for (int pass = 0; pass < L; ++pass) {
    for (int i = 0; i < L * L; ++i) A[i] = M0[i];
    for (int j = 0; j < L; ++j) A[row * L + j] = 1.0;
    for (int i = 0; i < L; ++i) x[i] = 0.0;
    x[row] = C.ntot[k];
    lu_factor(A, piv, L);
    lu_solve(A, piv, x, L);
    int nr = 0;
    for (int i = 1; i < L; ++i)
      if (x[i] > x[nr]) nr = i;
    if (nr == row) break;
    row = nr;
  }
  for (int i = 0; i < L; ++i) out[k * L + i] = x[i];
}

__global__ void k_copy_out(const ColDev* __restrict__ cols, double* const* nout) {
  const ColDev& C = cols[blockIdx.x];
  double* dst = nout[blockIdx.x];
  for (int i = threadIdx.x; i < C.N; i += blockDim.x) dst[i] = C.n[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
#define HIP_TRY(x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return set_err(NLTE_E_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_));       \
  } while (0)

extern "C" nlte_status nlte_zero_radiation_populations(nlte_column* col, double* n_dev,
                                                       hipStream_t s) {
  if (!col || !n_dev) return set_err(NLTE_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(column_ctx(col)->device));
  const ColDev& C = column_dev(col);
  k_zero_radiation<<<(C.nz + 63) / 64, 64, 0, s>>>(column_dev_ptr(col), n_dev);
  HIP_TRY(hipGetLastError());
  return NLTE_OK;
}

// ---------------------------------------------------------------------------
// driver pieces shared by the batch solve and the server
// ---------------------------------------------------------------------------
__global__ void k_gather_state(const ColDev* __restrict__ cols, ColState* __restrict__ out, int ncol) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncol) out[c] = *cols[c].st;
}

// After a batch solve: every column idle for later residual calls.
__global__ void k_idle_state(const ColDev* __restrict__ cols, int ncol) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncol) {
    ColState* st = cols[c].st;
    st->mode = kModeIdle;
    st->want_J = 0;
    st->rows_own = 0;
  }
}

namespace nlte {

nlte_status check_solve_opts(const nlte_solve_opts& o) {
  if (o.restart < 1 || o.restart > kMaxM) return set_err(NLTE_E_INVALID, "restart must be 1..%d", kMaxM);
  if (o.maxiter < 0 || o.max_krylov < 1 || o.max_krylov_total < 0 || o.max_halvings < 0 ||
      !(o.ftol >= 0) || !(o.rtol > 0) || !(o.eps_scale > 0) || o.init < 0 || o.init > 2 ||
      o.krylov_x0 < 0 || o.krylov_x0 > 1 || (o.launch & ~(NLTE_SOLVE_GRAPH | NLTE_SOLVE_TUNE)) ||
      (o.krylov_method != NLTE_KRYLOV_GMRES && o.krylov_method != NLTE_KRYLOV_BICGSTAB) ||
      (o.jv_method != NLTE_JV_FD && o.jv_method != NLTE_JV_TANGENT))
    return set_err(NLTE_E_INVALID, "invalid solve options");
  return NLTE_OK;
}

hipError_t solver_init(const ColDev* cols, int ncol, const double* const* n0, const double* const* J0,
                       const nlte_solve_opts& o, hipStream_t s) {
  InitArgs ia{o.ftol, o.rtol, 2.220446049250313e-16, o.eps_scale, o.maxiter, o.max_krylov,
              o.restart, o.max_halvings, 0, o.max_krylov_total, o.fp64_fallback, o.krylov_method,
              o.jv_method, o.krylov_x0};
  k_solver_init<<<ncol, kThreads, 0, s>>>(cols, n0, J0, ia);
  return hipGetLastError();
}

hipError_t solver_step(const ColDev* cols, const int* act, int n, int* done, hipStream_t s) {
  k_solver_step<<<n, kThreads, 0, s>>>(cols, act, done);
  return hipGetLastError();
}

hipError_t solver_gather(const ColDev* cols, int ncol, ColState* out, hipStream_t s) {
  k_gather_state<<<(ncol + 127) / 128, 128, 0, s>>>(cols, out, ncol);
  return hipGetLastError();
}

bool state_done(const ColState& st) { return st.phase == PH_DONE; }

// Radiation-free start of a column whose solver state was just initialised:
// its first evaluation point and its initial populations (the restart point
// of an FP64 fallback) become the radiation-free populations.
void zero_radiation_into(const ColDev* dcol, const ColDev& hc, hipStream_t s) {
  k_zero_radiation<<<(hc.nz + 63) / 64, 64, 0, s>>>(dcol, hc.eval_n);
  (void)hipMemcpyAsync(hc.n_init, hc.eval_n, (size_t)hc.N * sizeof(double), hipMemcpyDeviceToDevice, s);
}

void state_stats(const ColState& st, nlte_solve_stats* out) {
  out->status = st.phase == PH_DONE ? st.status : NLTE_E_NOCONV;
  out->newton_iters = st.newton_it;
  out->krylov_iters = st.krylov_total;
  out->f_calls = st.f_calls;
  out->stalls = st.stalls;
  out->precond_calls = st.precond_calls;
  out->rho_inf = st.rho_cur;
  out->dn_inf = st.dn_inf;
  out->precision = st.cur_prec;
  out->fp64_evals = st.fp64_evals;
}

}  // namespace nlte

namespace {
// Graph replay of a batch solve's step blocks: the capture stream, the graph
// of the current block shape and work lists, and two timing events of the
// shape tuner.
struct StepReplay {
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  int captures = 0;
  void drop() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~StepReplay() {
    drop();
    if (cap) hipStreamDestroy(cap);
    if (t0) hipEventDestroy(t0);
    if (t1) hipEventDestroy(t1);
  }
};

struct Batch {
  ColDev* cols = nullptr;       // device array of column descriptors
  Tile* tiles = nullptr;
  int4* rate = nullptr;
  int2* prec = nullptr;
  double** n0 = nullptr;
  double** J0 = nullptr;
  double** nout = nullptr;
  int* act = nullptr;
  ColState* states = nullptr;
  int* done = nullptr;
  int* done_host = nullptr;     // pinned
  int* gidx = nullptr;          // per-step mode lists (BatchWork::gidx, mlist, mcount)
  Tile* mlist = nullptr;
  int* mcount = nullptr;
  int ncol = 0, ntiles = 0, maxL = 0, any64 = 0, any32 = 0;
  ~Batch() {
    if (gidx) hipFree(gidx);
    if (mlist) hipFree(mlist);
    if (mcount) hipFree(mcount);
    if (cols) hipFree(cols);
    if (tiles) hipFree(tiles);
    if (rate) hipFree(rate);
    if (prec) hipFree(prec);
    if (n0) hipFree(n0);
    if (J0) hipFree(J0);
    if (nout) hipFree(nout);
    if (act) hipFree(act);
    if (states) hipFree(states);
    if (done) hipFree(done);
    if (done_host) hipHostFree(done_host);
  }
};
}  // namespace

extern "C" nlte_status nlte_solve_batch(nlte_ctx* ctx, nlte_column* const* cols, int32_t ncol,
                                        const double* const* n0_dev, const double* const* J0_dev,
                                        const nlte_solve_opts* opts, double* const* n_out_dev,
                                        nlte_solve_stats* stats, hipStream_t s) {
  if (!ctx || !cols || ncol <= 0 || !n_out_dev) return set_err(NLTE_E_INVALID, "bad arguments");
  nlte_solve_opts o;
  nlte_solve_opts_default(&o);
  if (opts) o = *opts;
  {
    const nlte_status vs = check_solve_opts(o);
    if (vs != NLTE_OK) return vs;
  }
  if (o.init == 0 && !n0_dev) return set_err(NLTE_E_INVALID, "init = 0 needs n0");
  HIP_TRY(hipSetDevice(ctx->device));
  Batch b;
  b.ncol = ncol;
  std::vector<ColDev> hc(ncol);
  std::vector<Tile> tiles;
  std::vector<int4> rate_w;
  std::vector<int2> prec_w;
  for (int c = 0; c < ncol; ++c) {
    if (!cols[c]) return set_err(NLTE_E_INVALID, "column %d is NULL", c);
    if (column_ctx(cols[c]) != ctx) return set_err(NLTE_E_INVALID, "column %d from another context", c);
    hc[c] = column_dev(cols[c]);
    b.maxL = std::max(b.maxL, hc[c].L);
    if (hc[c].prec == NLTE_FP64) b.any64 = 1; else b.any32 = 1;
    for (int d = 0; d < c; ++d)
      if (cols[d] == cols[c]) return set_err(NLTE_E_INVALID, "column %d appears twice", c);
  }
  std::vector<TileGroup> groups;
  const int nrate0 = build_work_lists(hc.data(), ncol, tiles, groups, rate_w, prec_w, b.maxL);
  b.ntiles = (int)tiles.size();
  HIP_TRY(hipMalloc(&b.cols, ncol * sizeof(ColDev)));
  HIP_TRY(hipMalloc(&b.tiles, tiles.size() * sizeof(Tile)));
  HIP_TRY(hipMalloc(&b.rate, std::max<size_t>(1, rate_w.size()) * sizeof(int4)));
  HIP_TRY(hipMalloc(&b.prec, std::max<size_t>(1, prec_w.size()) * sizeof(int2)));
  HIP_TRY(hipMemcpyAsync(b.rate, rate_w.data(), rate_w.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b.prec, prec_w.data(), prec_w.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  BatchWork bw;
  bw.cols = b.cols;
  bw.tiles = b.tiles;
  bw.rate_work = b.rate;
  bw.pb_work = b.prec;
  bw.ncol = ncol;
  bw.ntiles = b.ntiles;
  bw.nrate = (int)rate_w.size();
  bw.nrate0 = nrate0;
  bw.npb = (int)prec_w.size();
  bw.any64 = b.any64;
  bw.any32 = b.any32;
  bw.any_newton = 1;
  bw.any_tangent = o.jv_method == NLTE_JV_TANGENT;
  if (!set_groups(bw, groups)) return set_err(NLTE_E_INVALID, "too many tile groups");
  for (int c = 0; c < ncol; ++c) bw.maxnz = std::max(bw.maxnz, hc[c].nz);
  bw.fallback = o.fp64_fallback > 0 && b.any32;
  // per-step mode lists: each formal-solution launch starts with the waves
  // of the columns it evaluates
  std::vector<int> gidx;
  set_mode_groups(bw, tiles, ncol, gidx);
  HIP_TRY(hipMalloc(&b.gidx, ncol * sizeof(int)));
  HIP_TRY(hipMalloc(&b.mlist, 4 * std::max<size_t>(1, tiles.size()) * sizeof(Tile)));
  HIP_TRY(hipMalloc(&b.mcount, 4 * kMaxGroups * sizeof(int)));
  HIP_TRY(hipMemcpyAsync(b.gidx, gidx.data(), ncol * sizeof(int), hipMemcpyHostToDevice, s));
  bw.gidx = b.gidx;
  bw.mlist = b.mlist;
  bw.mcount = b.mcount;

  HIP_TRY(hipMalloc(&b.nout, ncol * sizeof(double*)));
  HIP_TRY(hipMalloc(&b.done, sizeof(int)));
  HIP_TRY(hipHostMalloc(&b.done_host, sizeof(int)));
  HIP_TRY(hipMemcpyAsync(b.cols, hc.data(), ncol * sizeof(ColDev), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b.tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b.nout, n_out_dev, ncol * sizeof(double*), hipMemcpyHostToDevice, s));
  if (o.init == 0) {
    HIP_TRY(hipMalloc(&b.n0, ncol * sizeof(double*)));
    HIP_TRY(hipMemcpyAsync(b.n0, n0_dev, ncol * sizeof(double*), hipMemcpyHostToDevice, s));
  }
  if (J0_dev) {
    HIP_TRY(hipMalloc(&b.J0, ncol * sizeof(double*)));
    HIP_TRY(hipMemcpyAsync(b.J0, J0_dev, ncol * sizeof(double*), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(hipMemsetAsync(b.done, 0, sizeof(int), s));
  InitArgs ia{o.ftol, o.rtol, 2.220446049250313e-16, o.eps_scale, o.maxiter, o.max_krylov,
              o.restart, o.max_halvings, o.init, o.max_krylov_total, o.fp64_fallback, o.krylov_method,
              o.jv_method, o.krylov_x0};
  k_solver_init<<<ncol, 256, 0, s>>>(b.cols, o.init == 0 ? b.n0 : nullptr, b.J0, ia);
  if (o.init == 2)
    for (int c = 0; c < ncol; ++c) zero_radiation_into(column_dev_ptr(cols[c]), hc[c], s);
  HIP_TRY(hipGetLastError());
  // every step evaluates one residual per active column; bound the step count
  const long max_steps = (long)(o.maxiter + 1) * (o.max_krylov + o.max_krylov / o.restart + o.max_halvings + 4) + 16;
  const int check_every = 4;
  const bool prof = ctx->prof_on != 0;
  // graph replay of the blocks of check_every steps (eager when profiling,
  // whose per-phase events sit between the launches)
  const bool use_graph = (o.launch & NLTE_SOLVE_GRAPH) && !prof;
  const bool tune = (o.launch & NLTE_SOLVE_TUNE) != 0;
  StepReplay G;
  if (use_graph) {
    HIP_TRY(residual_streams_init());
    HIP_TRY(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
  }
  if (tune) {
    HIP_TRY(hipEventCreate(&G.t0));
    HIP_TRY(hipEventCreate(&G.t1));
  }
  // waves per formal-solution workgroup: one (the four concurrent launches
  // of a residual call share the device best), or tried on blocks 1..6
  // (block 0 holds the first, preconditioned evaluations) in the order 1,
  // 2, 4, 4, 2, 1: the cost of a step falls as the batch's Newton phase
  // settles, and a palindromic order gives each shape the same mean
  // position, so a linear trend does not favour the shape tried last
  const int wpb_try[3] = {1, 2, 4};
  const int tune_order[6] = {0, 1, 2, 2, 1, 0};
  double tune_ms[3] = {0.0, 0.0, 0.0};
  int tune_next = tune ? 0 : 6;
  bw.formal_wpb = 1;
  std::vector<hipEvent_t> ev;
  if (prof) {
    ev.resize(7 * check_every);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  }
  long step = 0;
  long block = 0;
  *b.done_host = 0;
  int nlisted = ncol;
  std::vector<ColState> hst(ncol);
  HIP_TRY(hipMalloc(&b.act, ncol * sizeof(int)));
  HIP_TRY(hipMalloc(&b.states, ncol * sizeof(ColState)));
  nlte_status loop_st = NLTE_OK;
  auto launch_block = [&](hipStream_t st, bool with_events) -> hipError_t {
    for (int r = 0; r < check_every; ++r) {
      hipEvent_t* e = with_events ? &ev[7 * r] : nullptr;
      hipError_t he = launch_residual(bw, st, e);
      k_solver_step<<<bw.act ? bw.nact : ncol, kThreads, 0, st>>>(b.cols, bw.act, b.done);
      if (with_events) hipEventRecord(e[5], st);
      if (he == hipSuccess) he = hipGetLastError();
      if (he != hipSuccess) return he;
    }
    return hipSuccess;
  };
  while (step < max_steps) {
    const bool timing = block >= 1 && tune_next < 6;
    if (timing && bw.formal_wpb != wpb_try[tune_order[tune_next]]) {
      bw.formal_wpb = wpb_try[tune_order[tune_next]];
      G.drop();  // captured with another shape
    }
    if (timing) HIP_TRY(hipEventRecord(G.t0, s));
    hipError_t he = hipSuccess;
    if (use_graph) {
      if (!G.exec) {
        he = hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal);
        if (he == hipSuccess) {
          const hipError_t le = launch_block(G.cap, false);
          hipGraph_t g = nullptr;
          he = hipStreamEndCapture(G.cap, &g);
          G.graph = g;
          if (he == hipSuccess) he = le;
        }
        if (he == hipSuccess) he = hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0);
        G.captures += 1;
      }
      if (he == hipSuccess) he = hipGraphLaunch(G.exec, s);
    } else {
      he = launch_block(s, prof);
    }
    if (he != hipSuccess) {
      loop_st = set_err(NLTE_E_DEVICE, "solver launch failed: %s", hipGetErrorString(he));
      break;
    }
    if (timing) HIP_TRY(hipEventRecord(G.t1, s));
    step += check_every;
    block += 1;
    HIP_TRY(hipMemcpyAsync(b.done_host, b.done, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (timing) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, G.t0, G.t1));
      tune_ms[tune_order[tune_next]] += 0.5 * ms / check_every;
      if (++tune_next == 6) {
        int best = 0;
        for (int i = 1; i < 3; ++i)
          if (tune_ms[i] < tune_ms[best]) best = i;
        if (bw.formal_wpb != wpb_try[best]) {
          bw.formal_wpb = wpb_try[best];
          G.drop();
        }
      }
    }
    if (prof) {
      for (int r = 0; r < check_every; ++r) {
        float t[5], tf;
        for (int q = 0; q < 5; ++q) HIP_TRY(hipEventElapsedTime(&t[q], ev[7 * r + q], ev[7 * r + q + 1]));
        HIP_TRY(hipEventElapsedTime(&tf, ev[7 * r + 1], ev[7 * r + 6]));
        ctx->prof.steps += 1;
        ctx->prof.formal_launches += 2 * bw.ngroup * (bw.fallback ? 2 : 1);
        ctx->prof.formal_f_launches += bw.ngroup;
        ctx->prof.formal_f_ms += tf;
        ctx->prof.opacity_ms += t[0];
        ctx->prof.formal_ms += t[1];
        ctx->prof.depth_ms += t[2];
        ctx->prof.assemble_ms += t[3];
        ctx->prof.solver_ms += t[4];
      }
    }
    if (*b.done_host >= ncol) break;
    // Once a quarter of the listed columns has finished, list only the
    // columns still running, so that the launches of the tail of a batch
    // cover live work only (finished columns would just return).
    const int remaining = ncol - *b.done_host;
    if (remaining * 4 <= nlisted * 3) {
      HIP_TRY(solver_gather(b.cols, ncol, b.states, s));
      HIP_TRY(hipMemcpyAsync(hst.data(), b.states, ncol * sizeof(ColState), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      std::vector<int> live;
      for (int c = 0; c < ncol; ++c)
        if (!state_done(hst[c])) live.push_back(c);
      if (live.empty()) break;
      tiles.clear();
      groups.clear();
      rate_w.clear();
      prec_w.clear();
      int maxL_l = 0;
      const int nrate0_l = build_work_lists(hc.data(), ncol, tiles, groups, rate_w, prec_w, maxL_l,
                                            live.data(), (int)live.size());
      HIP_TRY(hipMemcpyAsync(b.tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(b.rate, rate_w.data(), rate_w.size() * sizeof(int4), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(b.prec, prec_w.data(), prec_w.size() * sizeof(int2), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(b.act, live.data(), live.size() * sizeof(int), hipMemcpyHostToDevice, s));
      bw.ntiles = (int)tiles.size();
      bw.nrate = (int)rate_w.size();
      bw.nrate0 = nrate0_l;
      bw.npb = (int)prec_w.size();
      set_groups(bw, groups);  // a subset of the groups checked above
      set_mode_groups(bw, tiles, ncol, gidx);
      HIP_TRY(hipMemcpyAsync(b.gidx, gidx.data(), ncol * sizeof(int), hipMemcpyHostToDevice, s));
      bw.maxnz = 0;
      for (int c : live) bw.maxnz = std::max(bw.maxnz, hc[c].nz);
      bw.act = b.act;
      bw.nact = (int)live.size();
      nlisted = (int)live.size();
      G.drop();  // the lists changed: capture again
      HIP_TRY(hipStreamSynchronize(s));  // host vectors are reused by the next rebuild
    }
  }
  ctx->prof.last_graph = use_graph ? 1 : 0;
  ctx->prof.last_formal_wpb = bw.formal_wpb;
  for (int i = 0; i < 3; ++i) ctx->prof.last_tune_ms[i] = tune_ms[i];
  ctx->prof.last_captures = G.captures;
  for (auto& e : ev) hipEventDestroy(e);
  if (loop_st != NLTE_OK) return loop_st;
  k_copy_out<<<ncol, 256, 0, s>>>(b.cols, b.nout);
  HIP_TRY(hipGetLastError());
  // final states in one copy, then every column idle for later residual calls
  std::vector<ColState> sts(ncol);
  HIP_TRY(solver_gather(b.cols, ncol, b.states, s));
  HIP_TRY(hipMemcpyAsync(sts.data(), b.states, ncol * sizeof(ColState), hipMemcpyDeviceToHost, s));
  k_idle_state<<<(ncol + 127) / 128, 128, 0, s>>>(b.cols, ncol);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  bool all_ok = true;
  for (int c = 0; c < ncol; ++c) {
    nlte_solve_stats one;
    state_stats(sts[c], &one);
    if (one.status != NLTE_OK) all_ok = false;
    if (stats) stats[c] = one;
  }
  if (!all_ok) {
    set_err(NLTE_E_NOCONV, "not every column converged (see stats)");
    return NLTE_E_NOCONV;
  }
  return NLTE_OK;
}

extern "C" nlte_status nlte_solve(nlte_column* col, const double* n0_dev, const double* J0_dev,
                                  const nlte_solve_opts* opts, double* n_out_dev, double* J_out_dev,
                                  nlte_solve_stats* stats, hipStream_t s) {
  if (!col || !n_out_dev) return set_err(NLTE_E_INVALID, "NULL argument");
  nlte_column* cols[1] = {col};
  const double* n0s[1] = {n0_dev};
  const double* J0s[1] = {J0_dev};
  double* outs[1] = {n_out_dev};
  nlte_status st = nlte_solve_batch(column_ctx(col), cols, 1, n0_dev ? n0s : nullptr,
                                    J0_dev ? J0s : nullptr, opts, outs, stats, s);
  if (J_out_dev && (st == NLTE_OK || st == NLTE_E_NOCONV)) {
    // the J-dagger of the final residual: with background scattering the
    // column's lagged J, otherwise (F does not depend on it) the final J
    const ColDev& C = column_dev(col);
    if (C.has_sca)
      HIP_TRY(hipMemcpyAsync(J_out_dev, C.Jdag, (size_t)C.nz * C.nnu * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    else
      transpose_J(C, J_out_dev, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
  }
  return st;
}
