// Residual F(n) on the device (Algorithm 1): opacity and emissivity assembly
// (Eqs. chi, eta), the short-characteristics formal solution for every
// frequency and ray (Eqs. Iplus, Iminus, App. A.1), the angle quadrature into
// the mean intensity, the frequency quadrature into radiative rates
// (Eqs. Rij, Rji), the rate-equation residual with conservation rows
// (Eqs. residuals_1, residuals_2) and, in Newton mode, the block-Jacobi
// preconditioner (Sect. 2.5.2 first solution, App. A.2).
//
// Work decomposition.
//   k_formal : one wavefront per chunk of 64 consecutive frequencies of one
//              column, one lane per frequency carrying all 2 x nmu rays
//              through the depth recursion in registers.  The first sweep
//              runs top -> bottom (ingoing rays) and parks their share of J
//              in a [k][nu] scratch row; the second runs bottom -> top
//              (outgoing rays) and writes J.  In Newton mode it also writes
//              the angle-averaged local intensity derivatives.
//   k_rates  : one lane per depth, one wavefront per (column, transition,
//              64 depths): each lane sums its transition window in frequency
//              order, so rate integrals need no cross-lane reductions and do
//              not depend on how columns are batched.
//   k_precond: Newton mode only; one lane per depth accumulates the
//              radiative part of the diagonal Jacobian blocks over a segment
//              of frequencies.
//   k_assemble: rates, rate-equation residual, conservation rows, scaled
//              residual, preconditioner blocks; one block per column.
#include "nlte_internal.h"

namespace nlte {

// ---------------------------------------------------------------------------
// piecewise-linear coefficients (Appendix A.1)
// ---------------------------------------------------------------------------

// e = exp(-x), a = 1 - (1 - e)/x, b = (1 - e)/x - e.  Below x = 0.1 (FP64)
// or 0.25 (FP32) a and b come from their Taylor series, which avoids the
// cancellation of the closed forms at small optical depth steps.
__device__ __forceinline__ void pl_coef(double x, double& e, double& a, double& b) {
  e = exp(-x);
  if (x < 0.1) {
    // a/x = sum_{m>=1} (-1)^{m+1} x^{m-1}/(m+1)!, b/x = sum_{m>=1} (-1)^{m+1} m x^{m-1}/(m+1)!
    double sa = -1.0 / 87178291200.0, sb = -13.0 / 87178291200.0;  // m = 13 (1/14!)
    sa = sa * x + 1.0 / 6227020800.0;  sb = sb * x + 12.0 / 6227020800.0;   // m = 12
    sa = sa * x - 1.0 / 479001600.0;   sb = sb * x - 11.0 / 479001600.0;    // m = 11
    sa = sa * x + 1.0 / 39916800.0;    sb = sb * x + 10.0 / 39916800.0;     // m = 10
    sa = sa * x - 1.0 / 3628800.0;     sb = sb * x - 9.0 / 3628800.0;       // m = 9
    sa = sa * x + 1.0 / 362880.0;      sb = sb * x + 8.0 / 362880.0;        // m = 8
    sa = sa * x - 1.0 / 40320.0;       sb = sb * x - 7.0 / 40320.0;         // m = 7
    sa = sa * x + 1.0 / 5040.0;        sb = sb * x + 6.0 / 5040.0;          // m = 6
    sa = sa * x - 1.0 / 720.0;         sb = sb * x - 5.0 / 720.0;           // m = 5
    sa = sa * x + 1.0 / 120.0;         sb = sb * x + 4.0 / 120.0;           // m = 4
    sa = sa * x - 1.0 / 24.0;          sb = sb * x - 3.0 / 24.0;            // m = 3
    sa = sa * x + 1.0 / 6.0;           sb = sb * x + 2.0 / 6.0;             // m = 2
    sa = sa * x - 0.5;                 sb = sb * x - 0.5;                   // m = 1 (sign)
    a = -sa * x;
    b = -sb * x;
  } else {
    const double t1 = (1.0 - e) / x;
    a = 1.0 - t1;
    b = t1 - e;
  }
}

__device__ __forceinline__ void pl_coef(float x, float& e, float& a, float& b) {
  e = __expf(-x);
  if (x < 0.25f) {
    float sa = 1.0f / 39916800.0f, sb = 10.0f / 39916800.0f;  // m = 10
    sa = sa * x - 1.0f / 3628800.0f;   sb = sb * x - 9.0f / 3628800.0f;
    sa = sa * x + 1.0f / 362880.0f;    sb = sb * x + 8.0f / 362880.0f;
    sa = sa * x - 1.0f / 40320.0f;     sb = sb * x - 7.0f / 40320.0f;
    sa = sa * x + 1.0f / 5040.0f;      sb = sb * x + 6.0f / 5040.0f;
    sa = sa * x - 1.0f / 720.0f;       sb = sb * x - 5.0f / 720.0f;
    sa = sa * x + 1.0f / 120.0f;       sb = sb * x + 4.0f / 120.0f;
    sa = sa * x - 1.0f / 24.0f;        sb = sb * x - 3.0f / 24.0f;
    sa = sa * x + 1.0f / 6.0f;         sb = sb * x + 2.0f / 6.0f;
    sa = sa * x - 0.5f;                sb = sb * x - 0.5f;
    a = -sa * x;
    b = -sb * x;
  } else {
    const float t1 = (1.0f - e) * __builtin_amdgcn_rcpf(x);
    a = 1.0f - t1;
    b = t1 - e;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------------
// opacity and emissivity, Eqs. chi and eta (FP64)
// ---------------------------------------------------------------------------
// Per wave: the line windows overlapping its chunk (uniform, scalar
// registers) and, per lane, the edges' cross-sections at its frequency
// (depth independent, registers).  Per depth and lane: the table values that
// change with depth, loaded one depth ahead of their use.
struct LineMeta {
  int lo, up, voff, wl;
  double g;
};

struct DepthVals {
  double B, E, Jd;
  double v[kMaxChunkLines];
};

struct WaveOpac {
  LineMeta lm[kMaxChunkLines];
  int loff[kMaxChunkLines];   // f - window start (per lane)
  unsigned amask;             // lane inside line window j
  int nl;
  int elo[kMaxEdges];         // edge lower levels (uniform)
  double alpha[kMaxEdges];    // edge cross-sections at f (0 outside the window)
  double gam;
};

__device__ __forceinline__ void wave_opac_init(WaveOpac& w, const ColDev& C, int chunk, int f) {
  const int l0 = uni(C.ch_lptr[chunk]);
  w.nl = uni(C.ch_lptr[chunk + 1]) - l0;
  w.amask = 0;
#pragma unroll
  for (int j = 0; j < kMaxChunkLines; ++j) {
    w.lm[j] = LineMeta{0, 0, 0, 0, 0.0};
    w.loff[j] = 0;
    if (j < w.nl) {
      const int t = uni(C.ch_line[l0 + j]);
      const TrDev& T = C.tr[t];
      const int wlo = uni(T.wlo), whi = uni(T.whi);
      w.lm[j] = LineMeta{uni(T.lo), uni(T.up), uni(T.voff), whi - wlo, uni(T.g)};
      w.loff[j] = f - wlo;
      if (f >= wlo && f < whi) w.amask |= 1u << j;
    }
  }
#pragma unroll
  for (int e = 0; e < kMaxEdges; ++e) {
    w.elo[e] = 0;
    w.alpha[e] = 0.0;
    if (e < C.nbf) {
      const TrDev& T = C.tr[C.nline + e];
      const int wlo = uni(T.wlo), whi = uni(T.whi);
      w.elo[e] = uni(T.lo);
      if (f >= wlo && f < whi) w.alpha[e] = ldg(C.V + uni(T.voff) + (f - wlo));
    }
  }
  w.gam = ldg(C.gam + f);
}

__device__ __forceinline__ void load_depth(DepthVals& d, const WaveOpac& w, const ColDev& C,
                                           int k, int f) {
  const size_t kf = (size_t)k * C.nnu + f;
  d.B = ldg(C.Bnu + kf);
  d.E = C.nbf ? ldg(C.Ebf + kf) : 0.0;
  d.Jd = C.has_sca ? ldg(C.Jdag + kf) : 0.0;
#pragma unroll
  for (int j = 0; j < kMaxChunkLines; ++j) {
    d.v[j] = 0.0;
    if (j < w.nl && ((w.amask >> j) & 1u))
      d.v[j] = ldg(C.V + w.lm[j].voff + (size_t)k * w.lm[j].wl + w.loff[j]);
  }
}

struct Opac {
  double chi, eta;
};

__device__ __forceinline__ Opac opacity(const WaveOpac& w, const DepthVals& d, const ColDev& C,
                                        const double* __restrict__ n, int k) {
  const int L = C.L;
  const double* nk = n + k * L;
  const double cc = ldc(C.chi_c + k), cs = ldc(C.chi_sca + k);
  Opac o;
  o.chi = cc + cs;
  o.eta = cc * d.B + cs * d.Jd;
  if (C.nbf) {
    // edges: V = alpha, g = (n*_l/n*_c) exp(-h nu/kT); sum_e alpha (n_l - g n_c)
    const double* rho = C.rho_bf + k * C.nbf;
    double A1 = 0.0, A2 = 0.0;
#pragma unroll
    for (int e = 0; e < kMaxEdges; ++e) {
      if (e < C.nbf) {
        A1 += w.alpha[e] * ldc(nk + w.elo[e]);
        A2 += w.alpha[e] * ldc(rho + e);
      }
    }
    const double nc = ldc(nk + L - 1);
    o.chi += A1 - d.E * nc * A2;
    o.eta += w.gam * d.E * nc * A2;
  }
#pragma unroll
  for (int j = 0; j < kMaxChunkLines; ++j) {
    if (j < w.nl) {
      const double nl_ = ldc(nk + w.lm[j].lo), nu_ = ldc(nk + w.lm[j].up);
      o.chi += d.v[j] * (nl_ - w.lm[j].g * nu_);
      o.eta += w.gam * w.lm[j].g * d.v[j] * nu_;
    }
  }
  return o;
}

// ---------------------------------------------------------------------------
// formal solution kernel
// ---------------------------------------------------------------------------
// R: arithmetic of the depth recursion (double, or float for the FP32 form).
// PM: Newton mode (also the local intensity derivatives of App. A.2).
// The first sweep assembles chi and S at every depth and keeps them in a
// [k][nu] scratch row for the second sweep, which only reloads them.
template <typename R, bool PM>
__device__ __forceinline__ void formal_tile(const ColDev& C, int chunk, int lane) {
  const int nz = C.nz, nnu = C.nnu, nmu = C.nmu;
  const int f = chunk * kWave + lane;
  const bool fin = f < nnu;
  const int fc = fin ? f : nnu - 1;
  const double* __restrict__ n = C.eval_n;
  R* __restrict__ xs = reinterpret_cast<R*>(C.XS);  // [nz][nnu][2]: chi, S

  WaveOpac w;
  wave_opac_init(w, C, chunk, fc);

  R wm2[kMaxMu], i2mu[kMaxMu];
#pragma unroll
  for (int m = 0; m < kMaxMu; ++m) {
    wm2[m] = (R)C.wm2[m];
    i2mu[m] = (R)C.inv2mu[m];
  }

  // ---- sweep 1: ingoing rays, top -> bottom (I- = 0 at the top) ----
  R I[kMaxMu];
#pragma unroll
  for (int m = 0; m < kMaxMu; ++m) I[m] = (R)0;
  R chi_p = 0, S_p = 0;
  DepthVals cur, nxt;
  load_depth(cur, w, C, 0, fc);
  for (int k = 0; k < nz; ++k) {
    if (k + 1 < nz) load_depth(nxt, w, C, k + 1, fc);
    const Opac o = opacity(w, cur, C, n, k);
    const R chi = (R)o.chi, S = (R)(o.eta / o.chi);
    double Jm = 0.0, dX = 0.0, dE = 0.0;
    if (k > 0) {
      const R dz = (R)ldc(C.dz + k - 1);
      const R base = dz * (chi_p + chi);
#pragma unroll
      for (int m = 0; m < kMaxMu; ++m) {
        if (m < nmu) {
          const R dt = base * i2mu[m];
          R e, a, b;
          pl_coef(dt, e, a, b);
          const R Iup = I[m];
          I[m] = Iup + a * (S - Iup) + b * (S_p - Iup);
          Jm += (double)wm2[m] * (double)I[m];
          if (PM) {
            // c_chi, c_eta of App. A.2 (ingoing ray, segment k-1 -> k)
            const R cchi = -(S / chi) * a +
                           dz * i2mu[m] * (e * (S_p - Iup) - (S_p - S) * b / dt);
            dX += (double)wm2[m] * (double)cchi;
            dE += (double)wm2[m] * (double)(a / chi);
          }
        }
      }
    }
    if (fin) {
      const size_t kf = (size_t)k * nnu + f;
      stg(C.Jm + kf, Jm);
      stg(xs + 2 * kf, chi);
      stg(xs + 2 * kf + 1, S);
      if (PM) {
        stg(C.Dchi + kf, dX);
        stg(C.Deta + kf, dE);
      }
    }
    chi_p = chi;
    S_p = S;
    cur = nxt;
  }

  // ---- sweep 2: outgoing rays, bottom -> top (I+ = B at the bottom) ----
  R chi_n = chi_p, S_n = S_p;
  {
    const size_t kf = (size_t)(nz - 1) * nnu + fc;
    const R Bb = (R)ldg(C.Bnu + kf);
    double Jp = 0.0;
#pragma unroll
    for (int m = 0; m < kMaxMu; ++m) {
      I[m] = Bb;
      if (m < nmu) Jp += (double)wm2[m] * (double)Bb;
    }
    if (fin) {
      const size_t fk = (size_t)f * nz + (nz - 1);
      stg(C.JT + fk, ldg(C.Jm + kf) + Jp);
      if (PM) {  // bottom: ingoing-ray derivatives only
        stg(C.DchiT + fk, ldg(C.Dchi + kf));
        stg(C.DetaT + fk, ldg(C.Deta + kf));
      }
    }
  }
  // prefetched: chi, S, Jm (and the ingoing derivatives) of the next depth up
  R chi_c = 0, S_c = 0;
  double Jm_c = 0.0, dX_c = 0.0, dE_c = 0.0;
  if (nz >= 2) {
    const size_t kf = (size_t)(nz - 2) * nnu + fc;
    chi_c = ldg(xs + 2 * kf);
    S_c = ldg(xs + 2 * kf + 1);
    Jm_c = ldg(C.Jm + kf);
    if (PM) {
      dX_c = ldg(C.Dchi + kf);
      dE_c = ldg(C.Deta + kf);
    }
  }
  for (int k = nz - 2; k >= 0; --k) {
    R chi_x = 0, S_x = 0;
    double Jm_x = 0.0, dX_x = 0.0, dE_x = 0.0;
    if (k > 0) {
      const size_t kf = (size_t)(k - 1) * nnu + fc;
      chi_x = ldg(xs + 2 * kf);
      S_x = ldg(xs + 2 * kf + 1);
      Jm_x = ldg(C.Jm + kf);
      if (PM) {
        dX_x = ldg(C.Dchi + kf);
        dE_x = ldg(C.Deta + kf);
      }
    }
    const R chi = chi_c, S = S_c;
    const R dz = (R)ldc(C.dz + k);
    const R base = dz * (chi + chi_n);
    double Jp = 0.0, dX = 0.0, dE = 0.0;
#pragma unroll
    for (int m = 0; m < kMaxMu; ++m) {
      if (m < nmu) {
        const R dt = base * i2mu[m];
        R e, a, b;
        pl_coef(dt, e, a, b);
        const R Iup = I[m];
        I[m] = Iup + a * (S - Iup) + b * (S_n - Iup);
        Jp += (double)wm2[m] * (double)I[m];
        if (PM) {
          // a_chi, a_eta of App. A.2 (outgoing ray, segment k+1 -> k)
          const R achi = -(S / chi) * a +
                         dz * i2mu[m] * (e * (S_n - Iup) - (S_n - S) * b / dt);
          dX += (double)wm2[m] * (double)achi;
          dE += (double)wm2[m] * (double)(a / chi);
        }
      }
    }
    if (fin) {
      const size_t fk = (size_t)f * nz + k;
      stg(C.JT + fk, Jm_c + Jp);
      if (PM) {
        stg(C.DchiT + fk, dX_c + dX);
        stg(C.DetaT + fk, dE_c + dE);
      }
    }
    chi_n = chi;
    S_n = S;
    chi_c = chi_x;
    S_c = S_x;
    Jm_c = Jm_x;
    dX_c = dX_x;
    dE_c = dE_x;
  }
}

// One launch covers every tile of a step; each wave takes the mode of its
// column (residual only, or residual + preconditioner derivatives).
template <typename R>
__global__ __launch_bounds__(256) void k_formal(const ColDev* __restrict__ cols,
                                                const Tile* __restrict__ tiles, int ntiles) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tid = blockIdx.x * (blockDim.x >> 6) + wave;
  if (tid >= ntiles) return;
  const int col = uni(tiles[tid].col);
  const int chunk = uni(tiles[tid].chunk);
  const ColDev& C = cols[col];
  const int mode = uni(C.st->mode);
  if (mode == kModeIdle) return;
  if ((C.prec == NLTE_FP32_FORM) != (sizeof(R) == sizeof(float))) return;
  if (mode == kModeNewton)
    formal_tile<R, true>(C, chunk, lane);
  else
    formal_tile<R, false>(C, chunk, lane);
}

// ---------------------------------------------------------------------------
// rate integrals (Eqs. Rij, Rji): one lane per depth, sequential sums over
// each transition window (depth-contiguous operands, so every load of a
// wave is one contiguous run).  Lines: sum cw V J.  Edges: sum cw alpha J and
// sum cw alpha exp(-h nu/kT) J (the J part of R_ul without its depth factor).
// Compensated (Neumaier) sums: windows run to thousands of points and the
// residual cancels gross rates, so plain sequential sums would set its floor.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
  const double u = s + x;
  c += (fabs(s) >= fabs(x)) ? (s - u) + x : (x - u) + s;
  s = u;
}

__device__ __forceinline__ void rates_item(const ColDev& C, int t, int k0) {
  if (uni(C.st->mode) == kModeIdle) return;
  const int nz = C.nz;
  const int k = k0 + threadIdx.x;
  if (k >= nz) return;
  const TrDev& T = C.tr[t];
  const int wlo = uni(T.wlo), wl = uni(T.whi) - wlo;
  const double* __restrict__ J = C.JT + (size_t)wlo * nz + k;
  const double* __restrict__ cw = C.cw + uni(T.cwoff);
  double* dst = C.RJ + ((size_t)k * C.ntr + t) * 2;
  if (t < C.nline) {
    const double* __restrict__ V = C.VT + uni(T.voff) + k;
    double s = 0.0, c = 0.0;
#pragma unroll 4
    for (int q = 0; q < wl; ++q)
      neumaier(s, c, cw[q] * ldg(V + (size_t)q * nz) * ldg(J + (size_t)q * nz));
    stg(dst, s + c);
    stg(dst + 1, 0.0);
  } else {
    const double* __restrict__ A = C.V + uni(T.voff);
    const double* __restrict__ E = C.EbfT + (size_t)wlo * nz + k;
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
#pragma unroll 4
    for (int q = 0; q < wl; ++q) {
      const double x = cw[q] * A[q] * ldg(J + (size_t)q * nz);
      neumaier(s1, c1, x);
      neumaier(s2, c2, x * ldg(E + (size_t)q * nz));
    }
    stg(dst, s1 + c1);
    stg(dst + 1, s2 + c2);
  }
}

// ---------------------------------------------------------------------------
// radiative part of the diagonal Jacobian blocks (Sect. 2.5.1, 2.5.2 first
// solution):  P_ij += sum_nu alpha_i (beta_j D_chi + gamma_j D_eta).
// alpha_i, beta_j and gamma_j are sums over the transitions touching a level,
// so the block is a sum over pairs of transitions (t, t') of
//   M1 = sum_nu cw_t A_t V_t' D_chi,
//   M2 = sum_nu cw_t A_t g_t' V_t' (2 h nu^3/c^2 D_eta - D_chi),
// over the intersection of their windows, A_t = V_t (n_l - g_t n_u); the
// assembly scatters M1, M2 to the levels.  One lane per depth.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tr_vg(const ColDev& C, int t, int voff, int wlo, double gline,
                                      int kk, int q, double E, double& V, double& g) {
  if (t < C.nline) {
    V = ldg(C.VT + voff + (size_t)(q - wlo) * C.nz + kk);
    g = gline;
  } else {
    V = C.V[voff + (q - wlo)];
    g = C.rho_bf[kk * C.nbf + (t - C.nline)] * E;
  }
}

__device__ __forceinline__ void precond_item(const ColDev& C, int p, int k0) {
  const int nz = C.nz, L = C.L;
  const int k = k0 + threadIdx.x;
  if (k >= nz) return;
  const int4 pr = C.pairs[p];
  const int t = uni(pr.x), u = uni(pr.y), f0 = uni(pr.z), f1 = uni(pr.w);
  const TrDev& Tt = C.tr[t];
  const TrDev& Tu = C.tr[u];
  const int tw = uni(Tt.wlo), uw = uni(Tu.wlo), tv = uni(Tt.voff), uv = uni(Tu.voff);
  const double tg = uni(Tt.g), ug = uni(Tu.g);
  const double* cwt = C.cw + uni(Tt.cwoff) - tw;
  const double nl = C.eval_n[k * L + uni(Tt.lo)], nu_ = C.eval_n[k * L + uni(Tt.up)];
  const bool edge = t >= C.nline || u >= C.nline;
  double m1 = 0.0, m2 = 0.0;
#pragma unroll 4
  for (int q = f0; q < f1; ++q) {
    const size_t fk = (size_t)q * nz + k;
    const double E = edge ? ldg(C.EbfT + fk) : 0.0;
    double Vt, gt, Vu, gu;
    tr_vg(C, t, tv, tw, tg, k, q, E, Vt, gt);
    tr_vg(C, u, uv, uw, ug, k, q, E, Vu, gu);
    const double DX = ldg(C.DchiT + fk), DE = ldg(C.DetaT + fk);
    const double cA = cwt[q] * Vt * (nl - gt * nu_);
    m1 += cA * Vu * DX;
    m2 += cA * gu * Vu * (C.gam[q] * DE - DX);
  }
  double* dst = C.M + ((size_t)k * C.npair + p) * 2;
  stg(dst, m1);
  stg(dst + 1, m2);
}

// Lane-per-depth work of a step: rate integrals (kind 0) of every active
// column and, for columns in Newton mode, preconditioner pair sums (kind 1).
__global__ __launch_bounds__(64) void k_depthwork(const ColDev* __restrict__ cols,
                                                  const int4* __restrict__ work, int nwork) {
  const int w = blockIdx.x;
  if (w >= nwork) return;
  const int4 it = work[w];
  const int col = uni(it.x), idx = uni(it.y), k0 = uni(it.z), kind = uni(it.w);
  const ColDev& C = cols[col];
  const int mode = uni(C.st->mode);
  if (kind == 0) {
    if (mode != kModeIdle) rates_item(C, idx, k0);
  } else {
    if (mode == kModeNewton) precond_item(C, idx, k0);
  }
}

// ---------------------------------------------------------------------------
// assembly: rates, F rows, conservation rows, rho, preconditioner blocks
// ---------------------------------------------------------------------------
constexpr int kAsmThreads = 128;

__global__ __launch_bounds__(kAsmThreads) void k_assemble(const ColDev* __restrict__ cols) {
  __shared__ double sF[kAsmThreads][kMaxLev + 1];
  __shared__ double sG[kAsmThreads][kMaxLev + 1];
  const ColDev& C = cols[blockIdx.x];
  const int mode = uni(C.st->mode);
  if (mode == kModeIdle) return;
  const int nz = C.nz, L = C.L, ntr = C.ntr, nline = C.nline;
  const int tx = threadIdx.x;
  double rmax = 0.0;
  for (int k = tx; k < nz; k += blockDim.x) {
    const double* nk = C.eval_n + k * L;
    double* Fk = sF[tx];
    double* Gk = sG[tx];
    for (int i = 0; i < L; ++i) {
      Fk[i] = 0.0;
      Gk[i] = 0.0;
    }
    for (int t = 0; t < ntr; ++t) {
      const TrDev& T = C.tr[t];
      const int lo = uni(T.lo), up = uni(T.up);
      const double* rj = C.RJ + ((size_t)k * ntr + t) * 2;
      const double Rlu = rj[0];
      const double Rsp = C.Rsp[k * ntr + t];
      const double Rul = (t < nline) ? uni(T.g) * (Rsp + Rlu)
                                     : C.rho_bf[k * C.nbf + (t - nline)] * (Rsp + rj[1]);
      double* R = C.R + ((size_t)k * ntr + t) * 2;
      R[0] = Rlu;
      R[1] = Rul;
      const double up_rate = C.C_lu[k * ntr + t] + Rlu;
      const double dn_rate = C.C_ul[k * ntr + t] + Rul;
      double* Rt = C.Rtot + ((size_t)k * ntr + t) * 2;
      Rt[0] = up_rate;
      Rt[1] = dn_rate;
      const double out_l = nk[lo] * up_rate;
      const double out_u = nk[up] * dn_rate;
      const double kap = out_l - out_u;
      Fk[lo] += kap;
      Fk[up] -= kap;
      const double gross = fabs(out_l) + fabs(out_u);
      Gk[lo] += gross;
      Gk[up] += gross;
    }
    int r;
    if (C.st->rows_own) {
      r = 0;
      double best = nk[0];
      for (int i = 1; i < L; ++i)
        if (nk[i] > best) {
          best = nk[i];
          r = i;
        }
    } else {
      r = C.rows_frozen[k];
    }
    C.rows[k] = r;
    double sum = 0.0;
    for (int i = 0; i < L; ++i) sum += nk[i];
    // keep the rate row that the conservation row replaces, so a caller can
    // move the conservation row without another formal solution
    C.Fsave[k] = Fk[r];
    C.Gsave[k] = Gk[r];
    Fk[r] = C.ntot[k] - sum;
    Gk[r] = C.ntot[k];
    double rk = 0.0;
    for (int i = 0; i < L; ++i) {
      C.F[k * L + i] = Fk[i];
      C.G[k * L + i] = Gk[i];
      const double q = fabs(Fk[i]) / Gk[i];
      rk = (q > rk || q != q) ? q : rk;
    }
    C.rho_k[k] = rk;
    rmax = (rk > rmax || rk != rk) ? rk : rmax;
  }
  // block max (NaN-propagating)
  __shared__ double sm[kAsmThreads];
  sm[tx] = rmax;
  __syncthreads();
  for (int o = kAsmThreads / 2; o > 0; o >>= 1) {
    if (tx < o) {
      const double a = sm[tx], b = sm[tx + o];
      sm[tx] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  if (tx == 0) C.st->rho_eval = sm[0];
}

// Preconditioner blocks of Newton-mode columns: one thread per (depth, entry)
// gathers its contributions (Gamma from the total rates, the radiative part
// from the pair sums) from a per-column list, then the conservation row of
// the depth becomes -1 (the original row is kept in Psave).
__global__ __launch_bounds__(256) void k_pblock(const ColDev* __restrict__ cols,
                                                const int2* __restrict__ work, int nwork) {
  const int w = blockIdx.x;
  if (w >= nwork) return;
  const int col = uni(work[w].x), base = uni(work[w].y);
  const ColDev& C = cols[col];
  if (uni(C.st->mode) != kModeNewton) return;
  const int L = C.L, LL = L * L;
  const int id = base + threadIdx.x;
  if (id >= C.nz * LL) return;
  const int k = id / LL, ij = id - k * LL;
  const int i = ij / L, j = ij - i * L;
  const double* Rt = C.Rtot + (size_t)k * C.ntr * 2;
  const double* Mk = C.M + (size_t)k * C.npair * 2;
  double s = 0.0;
  for (int e = C.pg_ptr[ij]; e < C.pg_ptr[ij + 1]; ++e) {
    const int code = C.pg_code[e];
    const int kind = (code >> 1) & 3, idx = code >> 3;
    const double v = kind < 2 ? Rt[idx * 2 + kind] : Mk[idx * 2 + (kind - 2)];
    s += (code & 1) ? -v : v;
  }
  const int r = C.rows[k];
  if (i == r) {
    C.Psave[k * L + j] = s;
    s = -1.0;
  }
  C.P[(size_t)k * LL + ij] = s;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
hipError_t launch_residual(const BatchWork& bw, hipStream_t s, hipEvent_t* ev) {
  const int blocks = (bw.ntiles + 3) / 4;
  if (ev) hipEventRecord(ev[0], s);
  if (bw.ntiles > 0) {
    if (bw.any64) k_formal<double><<<blocks, 256, 0, s>>>(bw.cols, bw.tiles, bw.ntiles);
    if (bw.any32) k_formal<float><<<blocks, 256, 0, s>>>(bw.cols, bw.tiles, bw.ntiles);
  }
  if (ev) hipEventRecord(ev[1], s);
  if (bw.nrate > 0) k_depthwork<<<bw.nrate, 64, 0, s>>>(bw.cols, bw.rate_work, bw.nrate);
  if (ev) hipEventRecord(ev[2], s);
  k_assemble<<<bw.ncol, kAsmThreads, 0, s>>>(bw.cols);
  if (bw.any_newton && bw.npb > 0) k_pblock<<<bw.npb, 256, 0, s>>>(bw.cols, bw.pb_work, bw.npb);
  if (ev) hipEventRecord(ev[3], s);
  return hipGetLastError();
}

// Work lists of a batch (host side): formal-solution tiles, rate items and
// preconditioner items for every column.
void build_work_lists(const ColDev* hc, int ncol, std::vector<Tile>& tiles,
                      std::vector<int4>& rate, std::vector<int2>& pblock, int& maxL) {
  // rate items (kind 0) and preconditioner pair items (kind 1) share one list
  maxL = 0;
  for (int c = 0; c < ncol; ++c)
    for (int b = 0; b < hc[c].nz * hc[c].L * hc[c].L; b += 256) pblock.push_back(make_int2(c, b));
  for (int c = 0; c < ncol; ++c) {
    const ColDev& C = hc[c];
    maxL = std::max(maxL, C.L);
    for (int ch = 0; ch < C.nchunk; ++ch) tiles.push_back(Tile{c, ch});
    for (int t = 0; t < C.ntr; ++t)
      for (int k0 = 0; k0 < C.nz; k0 += kWave) rate.push_back(make_int4(c, t, k0, 0));
    for (int p = 0; p < C.npair; ++p)
      for (int k0 = 0; k0 < C.nz; k0 += kWave) rate.push_back(make_int4(c, p, k0, 1));
  }
}

}  // namespace nlte
