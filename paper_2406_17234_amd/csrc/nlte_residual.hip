// Residual F(n) on the device (Algorithm 1): opacity and emissivity assembly
// (Eqs. chi, eta), the short-characteristics formal solution for every
// frequency and ray (Eqs. Iplus, Iminus, App. A.1), the angle quadrature into
// the mean intensity, the frequency quadrature into radiative rates
// (Eqs. Rij, Rji), the rate-equation residual with conservation rows
// (Eqs. residuals_1, residuals_2) and, in Newton mode, the block-Jacobi
// preconditioner (Sect. 2.5.2 first solution, App. A.2).
//
// Work decomposition.  One wavefront owns a chunk of 64 consecutive
// frequencies of one column; each lane owns one frequency and carries all
// 2 x nmu rays of it through the depth recursion in registers.  The first
// sweep runs top -> bottom for the ingoing rays and parks their share of J
// in a per-(k, nu) scratch row; the second sweep runs bottom -> top for the
// outgoing rays, completes J at each depth and immediately folds it into the
// chunk's partial rate sums (wave reductions), so J never has to be re-read
// from memory to form the rates.  The assembly kernel adds the partial sums of
// every chunk in a fixed order (results do not depend on how columns are
// batched) and builds F.
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
// opacity and emissivity at one (k, f), Eqs. chi and eta (FP64)
// ---------------------------------------------------------------------------
struct Opac {
  double chi, eta;
};

__device__ __forceinline__ Opac opacity_at(const ColDev& C, const double* __restrict__ n,
                                           int k, int f, int e0, int e1) {
  const int nnu = C.nnu, L = C.L;
  const size_t kf = (size_t)k * nnu + f;
  Opac o;
  o.chi = C.chi_c[k] + C.chi_sca[k];
  o.eta = C.chi_c[k] * C.Bnu[kf];
  if (C.has_sca) o.eta += C.chi_sca[k] * C.Jdag[kf];
  const double Ekf = C.nbf ? C.Ebf[kf] : 0.0;
  const double gam = C.gam[f];
  for (int e = e0; e < e1; ++e) {
    const TrDev T = C.tr[C.ch_tr[e]];
    if (f < T.wlo || f >= T.whi) continue;
    const int t = C.ch_tr[e];
    const double nl = n[k * L + T.lo], nu_ = n[k * L + T.up];
    double V, g;
    if (t < C.nline) {
      V = C.V[T.voff + (size_t)k * (T.whi - T.wlo) + (f - T.wlo)];
      g = T.g;
    } else {
      V = C.V[T.voff + (f - T.wlo)];
      g = C.rho_bf[k * C.nbf + (t - C.nline)] * Ekf;
    }
    o.chi += V * (nl - g * nu_);
    o.eta += gam * g * V * nu_;
  }
  return o;
}

// ---------------------------------------------------------------------------
// fused formal-solution kernel
// ---------------------------------------------------------------------------
// R: arithmetic of the depth recursion (double, or float for the FP32 form).
// PM: Newton mode (also the preconditioner's radiative blocks and J output).
template <typename R, bool PM>
__global__ __launch_bounds__(256) void k_formal(const ColDev* __restrict__ cols,
                                                const Tile* __restrict__ tiles, int ntiles) {
  extern __shared__ double lds[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tid = blockIdx.x * (blockDim.x >> 6) + wave;
  if (tid >= ntiles) return;
  const Tile tl = tiles[tid];
  const ColDev& C = cols[tl.col];
  const int mode = C.st->mode;
  if (mode == kModeIdle || (mode == kModeNewton) != PM) return;
  if ((C.prec == NLTE_FP32_FORM) != (sizeof(R) == sizeof(float))) return;
  const bool wantJ = PM || C.st->want_J;

  const int nz = C.nz, nnu = C.nnu, nmu = C.nmu, L = C.L;
  const int f = tl.chunk * kWave + lane;
  const bool fin = f < nnu;
  const int fc = fin ? f : nnu - 1;
  const double* __restrict__ n = C.eval_n;
  const int e0 = C.ch_ptr[tl.chunk], e1 = C.ch_ptr[tl.chunk + 1];

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
  for (int k = 0; k < nz; ++k) {
    const Opac o = opacity_at(C, n, k, fc, e0, e1);
    const R chi = (R)o.chi, S = (R)(o.eta / o.chi);
    double Jm = 0.0, dX = 0.0, dE = 0.0;
    if (k > 0) {
      const R dz = (R)C.dz[k - 1];
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
      C.Jm[(size_t)k * nnu + f] = Jm;
      if (PM) {
        C.Dchi[(size_t)k * nnu + f] = dX;
        C.Deta[(size_t)k * nnu + f] = dE;
      }
    }
    chi_p = chi;
    S_p = S;
  }

  // ---- sweep 2: outgoing rays, bottom -> top (I+ = B at the bottom) ----
  double* sA = nullptr;
  double* sX = nullptr;
  if (PM) {
    sA = lds + (size_t)wave * 2 * kWave * L;
    sX = sA + (size_t)kWave * L;
  }
  R chi_n = 0, S_n = 0;
  for (int k = nz - 1; k >= 0; --k) {
    const Opac o = opacity_at(C, n, k, fc, e0, e1);
    const R chi = (R)o.chi, S = (R)(o.eta / o.chi);
    const size_t kf = (size_t)k * nnu + fc;
    double Jp = 0.0, dX = 0.0, dE = 0.0;
    if (k == nz - 1) {
      const R Bb = (R)C.Bnu[kf];
#pragma unroll
      for (int m = 0; m < kMaxMu; ++m) {
        I[m] = Bb;
        if (m < nmu) Jp += (double)wm2[m] * (double)Bb;
      }
    } else {
      const R dz = (R)C.dz[k];
      const R base = dz * (chi + chi_n);
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
    }
    chi_n = chi;
    S_n = S;
    const double J = C.Jm[kf] + Jp;
    if (wantJ && fin) C.Jeval[kf] = J;

    // frequency quadrature: partial rate sums of this chunk
    const double Ekf = C.nbf ? C.Ebf[kf] : 0.0;
    for (int e = e0; e < e1; ++e) {
      const int t = C.ch_tr[e];
      const TrDev T = C.tr[t];
      const bool act = fin && f >= T.wlo && f < T.whi;
      double v1 = 0.0;
      if (act) {
        const double V = (t < C.nline) ? C.V[T.voff + (size_t)k * (T.whi - T.wlo) + (f - T.wlo)]
                                       : C.V[T.voff + (f - T.wlo)];
        v1 = C.cw[T.cwoff + (f - T.wlo)] * V * J;
      }
      const double s1 = wave_sum(v1);
      double* dst = C.part + ((size_t)C.ch_slot[e] * nz + k) * 2;
      if (t < C.nline) {
        if (lane == 0) dst[0] = s1;
      } else {
        const double s2 = wave_sum(v1 * Ekf);
        if (lane == 0) {
          dst[0] = s1;
          dst[1] = s2;
        }
      }
    }

    if (PM) {
      // Radiative block sum_f alpha_i (beta_j Dchi + gamma_j Deta) of this chunk.
      const double DX = (fin ? C.Dchi[kf] : 0.0) + dX;
      const double DE = (fin ? C.Deta[kf] : 0.0) + dE;
      double* a_l = sA + lane * L;
      double* x_l = sX + lane * L;
      for (int i = 0; i < L; ++i) {
        a_l[i] = 0.0;
        x_l[i] = 0.0;
      }
      if (fin) {
        const double gam = C.gam[f];
        for (int e = e0; e < e1; ++e) {
          const int t = C.ch_tr[e];
          const TrDev T = C.tr[t];
          if (f < T.wlo || f >= T.whi) continue;
          double V, g;
          if (t < C.nline) {
            V = C.V[T.voff + (size_t)k * (T.whi - T.wlo) + (f - T.wlo)];
            g = T.g;
          } else {
            V = C.V[T.voff + (f - T.wlo)];
            g = C.rho_bf[k * C.nbf + (t - C.nline)] * Ekf;
          }
          const double cA = C.cw[T.cwoff + (f - T.wlo)] * V * (n[k * L + T.lo] - g * n[k * L + T.up]);
          a_l[T.lo] += cA;
          a_l[T.up] -= cA;
          x_l[T.lo] += V * DX;
          x_l[T.up] += g * V * (gam * DE - DX);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double* dstP = C.Ppart + ((size_t)tl.chunk * nz + k) * L * L;
      for (int p = lane; p < L * L; p += kWave) {
        const int i = p / L, j = p - i * L;
        double s = 0.0;
        for (int q = 0; q < kWave; ++q) s += sA[q * L + i] * sX[q * L + j];
        dstP[p] = s;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// ---------------------------------------------------------------------------
// assembly: rates from the partial sums, F rows, conservation rows, rho,
// preconditioner blocks (Gamma + radiative part)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_assemble(const ColDev* __restrict__ cols) {
  __shared__ double sF[kWave][kMaxLev + 1];
  __shared__ double sG[kWave][kMaxLev + 1];
  const ColDev& C = cols[blockIdx.x];
  const int mode = C.st->mode;
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
    double* Pk = C.P + (size_t)k * L * L;
    if (mode == kModeNewton) {
      for (int p = 0; p < L * L; ++p) {
        double s = 0.0;
        for (int c = 0; c < C.nchunk; ++c) s += C.Ppart[((size_t)c * nz + k) * L * L + p];
        Pk[p] = s;
      }
    }
    for (int t = 0; t < ntr; ++t) {
      const TrDev T = C.tr[t];
      const int nch = chunk_of(T.whi - 1) - T.c0 + 1;
      double s1 = 0.0, s2 = 0.0;
      for (int s = 0; s < nch; ++s) {
        const double* src = C.part + ((size_t)(T.slot + s) * nz + k) * 2;
        s1 += src[0];
        if (t >= nline) s2 += src[1];
      }
      const double Rlu = s1;
      const double Rsp = C.Rsp[k * ntr + t];
      const double Rul = (t < nline) ? T.g * (Rsp + Rlu)
                                     : C.rho_bf[k * C.nbf + (t - nline)] * (Rsp + s2);
      C.R[((size_t)k * ntr + t) * 2 + 0] = Rlu;
      C.R[((size_t)k * ntr + t) * 2 + 1] = Rul;
      const double up_rate = C.C_lu[k * ntr + t] + Rlu;
      const double dn_rate = C.C_ul[k * ntr + t] + Rul;
      const double out_l = nk[T.lo] * up_rate;
      const double out_u = nk[T.up] * dn_rate;
      const double kap = out_l - out_u;
      Fk[T.lo] += kap;
      Fk[T.up] -= kap;
      const double gross = fabs(out_l) + fabs(out_u);
      Gk[T.lo] += gross;
      Gk[T.up] += gross;
      if (mode == kModeNewton) {
        // Gamma_ij = delta_ij sum_p (C_ip + R_ip) - (C_ji + R_ji)
        Pk[T.lo * L + T.lo] += up_rate;
        Pk[T.up * L + T.up] += dn_rate;
        Pk[T.lo * L + T.up] -= dn_rate;
        Pk[T.up * L + T.lo] -= up_rate;
      }
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
    if (mode == kModeNewton)
      for (int j = 0; j < L; ++j) {
        C.Psave[k * L + j] = Pk[r * L + j];
        Pk[r * L + j] = -1.0;
      }
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
  __shared__ double sm[64];
  sm[tx] = rmax;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if (tx < o) {
      const double a = sm[tx], b = sm[tx + o];
      sm[tx] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  if (tx == 0) C.st->rho_eval = sm[0];
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
size_t formal_pm_lds_bytes(int maxL) { return (size_t)4 * 2 * kWave * maxL * sizeof(double); }

hipError_t launch_residual(const ColDev* cols_dev, int ncol, const Tile* tiles_dev, int ntiles,
                           int any_fp64, int any_fp32, int any_newton, int maxL, hipStream_t s,
                           hipEvent_t* ev) {
  const int blocks = (ntiles + 3) / 4;
  if (ev) hipEventRecord(ev[0], s);
  if (ntiles > 0) {
    if (any_fp64) k_formal<double, false><<<blocks, 256, 0, s>>>(cols_dev, tiles_dev, ntiles);
    if (any_fp32) k_formal<float, false><<<blocks, 256, 0, s>>>(cols_dev, tiles_dev, ntiles);
  }
  if (ev) hipEventRecord(ev[1], s);
  if (ntiles > 0 && any_newton) {
    const size_t lds = formal_pm_lds_bytes(maxL);
    if (any_fp64) k_formal<double, true><<<blocks, 256, lds, s>>>(cols_dev, tiles_dev, ntiles);
    if (any_fp32) k_formal<float, true><<<blocks, 256, lds, s>>>(cols_dev, tiles_dev, ntiles);
  }
  if (ev) hipEventRecord(ev[2], s);
  k_assemble<<<ncol, 64, 0, s>>>(cols_dev);
  if (ev) hipEventRecord(ev[3], s);
  return hipGetLastError();
}

}  // namespace nlte
