// Columns with a velocity field (Sect. 3.5): each ray sees the line profiles
// Doppler-shifted by the velocity along it, so the opacity, the source
// function and the formal solution are per ray, the line rates keep the
// angle integral inside the frequency sum (Eqs. Rij, Rji) and the
// preconditioner's local blocks take each ray's own intensity derivatives
// (App. A.2).  FP64 or the FP32 form, sequential formal solution.  The other residual
// launches (level coefficients, edge rates, assembly, block gather) are
// those of nlte_residual.hip.
#include "nlte_kernels.h"

namespace nlte {

// ---------------------------------------------------------------------------
// formal solution with a velocity field (Sect. 3.5)
// ---------------------------------------------------------------------------
// Each ray sees the line profiles Doppler-shifted by the velocity along it,
// so chi and S differ from ray to ray and every ray carries its own through
// the recursion.  FP64; one wave per 64-frequency chunk, one lane per
// frequency, as k_formal.  The ray-independent part of the opacity
// (background, edges, scattering) is made once per depth in the first sweep
// and kept in XS for the second; each ray adds its line part from its own V
// table.  The line rates need the angle integral inside the frequency sum
// (sum_nu cw sum_rays (w_m/2) V_ray I_ray, Eqs. Rij, Rji), so the kernel
// takes them itself while every ray's intensity is in registers: per depth
// and line window covering the chunk, a fixed-order wave sum over the
// chunk's 64 frequencies gives one rate entry per (line, chunk); the
// ingoing sweep parks its half in the entry's second slot and the outgoing
// sweep completes it (deterministic, independent of batching; the edges'
// rates are the static sums over J).  Outputs: J (depth-contiguous, staged
// through LDS as in k_formal), the line rate entries and in Newton mode the
// local derivatives of every ray's intensity (App. A.2, one per ray: the
// preconditioner weighs them with the ray's own profiles).  Every lane of
// the last chunk computes (its frequency clamped into the grid) and stores
// into the padded rows, so no store needs a guard; its lanes beyond the grid
// add nothing to the rates.

// Wave-wide sum in a fixed butterfly order: lane 0's value is the same for
// every launch.
__device__ __forceinline__ double wave_sum0(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Line rate entries of depth k from the NMU rays r0 .. r0 + NMU - 1 of one
// sweep: per line window covering the chunk, sum over the chunk's
// frequencies of cw sum_m (w_m/2) V_ray I_ray.  The ingoing sweep (first)
// parks its sum in the entry's second slot; the outgoing sweep adds its own
// and writes the entry (second slot back to zero, as for every line entry).
template <int NMU, typename R>
__device__ __forceinline__ void vel_rate_step(const ColDev& C, int chunk, int k, int f, int fc,
                                              int r0, const R (&I)[NMU], const double (&wm2)[NMU],
                                              bool first) {
  const int nz = C.nz, nray = C.nray, nnu = C.nnu;
  const int l0 = ldc(C.ch_lptr + chunk), l1 = ldc(C.ch_lptr + chunk + 1);
  double* row = C.RJ + (size_t)k * C.nrseg * 2;
  for (int j = l0; j < l1; ++j) {
    const int t = ldc(C.ch_line + j);
    const TrDev* T = C.tr + t;
    const int wlo = ldc(&T->wlo), wl = ldc(&T->whi) - wlo;
    const int q = fc - wlo;
    const bool in = f < nnu && q >= 0 && q < wl;
    const size_t rstep = (size_t)nz * wl;
    const double* vr = C.VR + (size_t)nray * ldc(&T->voff) + (size_t)r0 * rstep + (size_t)k * wl + (in ? q : 0);
    double u = 0.0;
#pragma unroll
    for (int m = 0; m < NMU; ++m) u = fmar(wm2[m] * ldg(vr + m * rstep), (double)I[m], u);
    const double x = in ? ldg(C.cw + ldc(&T->cwoff) + q) * u : 0.0;
    const double tot = wave_sum0(x);
    if ((threadIdx.x & 63) == 0) {
      double* ent = row + 2 * (ldc(&T->sfirst) + chunk - wlo / kWave);
      if (first) {
        stg(ent + 1, tot);
      } else {
        stg(ent, ldg(ent + 1) + tot);
        stg(ent + 1, 0.0);
      }
    }
  }
}

// Ray-independent chi and eta at (k, fc): background, edges, scattering.
__device__ __forceinline__ void vel_base(const ColDev& C, int chunk, int k, int fc, double& chi0,
                                         double& eta0) {
  const int nz = C.nz, ntr = C.ntr;
  const double* __restrict__ coef = (const double*)C.coef;
  double A1 = 0.0, A2 = 0.0;
  const int e0 = ldc(C.ch_eptr + chunk), e1 = ldc(C.ch_eptr + chunk + 1);
  for (int j = e0; j < e1; ++j) {
    const int t = ldc(C.ch_edge + j);
    const TrDev* T = C.tr + t;
    const int wlo = ldc(&T->wlo), whi = ldc(&T->whi);
    const double al = (fc >= wlo && fc < whi) ? ldg(C.V + ldc(&T->voff) + (fc - wlo)) : 0.0;
    const double* ct = coef + ((size_t)t * nz + k) * 2;
    A1 = fmar(al, ldc(ct), A1);
    A2 = fmar(al, ldc(ct + 1), A2);
  }
  const size_t kf = (size_t)k * C.nnu + fc;
  const double E = C.nbf ? ldg(C.Ebf + kf) : 0.0;
  const double EA2 = E * A2;
  const double* cb = coef + ((size_t)ntr * nz + k) * 2;
  chi0 = ldc(cb) + (A1 - EA2);
  eta0 = fmar(ldc(cb + 1), ldg(C.EC + kf), ldg(C.gam + fc) * EA2);
  if (C.has_sca) eta0 = fmar(ldc(coef + ((size_t)(ntr + 1) * nz + k) * 2), ldg(C.Jdag + kf), eta0);
}

// chi and S at (k, fc) of the NMU rays r0 .. r0 + NMU - 1: the lines'
// V c0 and V c1 with each ray's V added to the ray-independent part.
template <int NMU, typename R>
__device__ __forceinline__ void vel_rays(const ColDev& C, int chunk, int k, int fc, double chi0,
                                         double eta0, int r0, R (&chi)[NMU], R (&S)[NMU]) {
  const int nz = C.nz, nray = C.nray;
  const double* __restrict__ coef = (const double*)C.coef;
  double cl[NMU], el[NMU];
#pragma unroll
  for (int m = 0; m < NMU; ++m) cl[m] = el[m] = 0.0;
  const int l0 = ldc(C.ch_lptr + chunk), l1 = ldc(C.ch_lptr + chunk + 1);
  for (int j = l0; j < l1; ++j) {
    const int t = ldc(C.ch_line + j);
    const TrDev* T = C.tr + t;
    const int wlo = ldc(&T->wlo), wl = ldc(&T->whi) - wlo;
    const int q = fc - wlo;
    const bool in = q >= 0 && q < wl;
    const double* ct = coef + ((size_t)t * nz + k) * 2;
    const double c0 = ldc(ct), c1 = ldc(ct + 1);
    const size_t rstep = (size_t)nz * wl;
    const double* vr = C.VR + (size_t)nray * ldc(&T->voff) + (size_t)r0 * rstep + (size_t)k * wl + (in ? q : 0);
    double v[NMU];
#pragma unroll
    for (int m = 0; m < NMU; ++m) v[m] = ldg(vr + m * rstep);
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      const double vi = in ? v[m] : 0.0;
      cl[m] = fmar(vi, c0, cl[m]);
      el[m] = fmar(vi, c1, el[m]);
    }
  }
  const double gam = ldg(C.gam + fc);
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    // the sums in FP64; only chi and S leave rounded to the recursion's
    // precision (as in the static FP32 form)
    const double X = chi0 + cl[m];
    chi[m] = (R)X;
    S[m] = (R)(fmar(gam, el[m], eta0) / X);
  }
}

// LDS per wave of the velocity formal solution: the J tile of KFV depths
// and, in Newton mode, one tile of KDV depths per ray and derivative.
constexpr int KFV = 8, KDV = 4;
template <bool PM, int NMU> struct VelStage {
  static constexpr int doubles = (KFV + (PM ? 2 * NMU * KDV : 0)) * kWave;
};

// R: the recursion's precision (double, or float for the FP32 form: chi and
// S rounded from their FP64 sums, the depth recursion in FP32, the angle
// sums into J, the rates and the derivatives' storage in FP64).
template <typename R, bool PM, int NMU>
__device__ __forceinline__ void formal_tile_vel(const ColDev& C, int chunk, int lane, double* tile) {
  constexpr int KF = KFV, KD = KDV;
  double* tJ = tile;
  double* tX = tile + KF * kWave;            // [NMU][KD * 64] per-ray D_chi
  double* tE = tX + NMU * KD * kWave;        // [NMU][KD * 64] per-ray D_eta
  const int nz = C.nz, nnu = C.nnu, fp = C.fp, zp = C.zp;
  const int f0 = chunk * kWave, f = f0 + lane;
  const int fc = f < nnu ? f : nnu - 1;
  const double* __restrict__ dzt = (const double*)C.coef + ((size_t)(C.ntr + 1) * nz) * 2 + 1;  // stride 2
  double* __restrict__ xb = C.XS;  // [nz][fp][2] ray-independent chi, eta
  double* __restrict__ jm = C.Jm;  // [nz][fp] ingoing half of J
  const size_t rs = (size_t)nnu * zp;  // ray stride of DXR, DER ([nray][nnu][zp])
  R i2mu[NMU], mu2[NMU];
  double wm2[NMU];
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    i2mu[m] = (R)C.inv2mu[m];
    mu2[m] = (R)(1.0 / C.inv2mu[m]);
    wm2[m] = C.wm2[m];
  }
  R I[NMU], chp[NMU], Sp[NMU], ch[NMU], Sx[NMU];
  // one segment of every ray of a sweep, from (chp, Sp) to (ch, Sx); returns
  // the rays' share of J and leaves the local derivatives in the tiles
  auto step = [&](int k, R dz) {
    double js = 0.0;
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      const R base = dz * (chp[m] + ch[m]);
      R e, q, a, bx;
      seg_coef<R, PM>(base * i2mu[m], PL<R>::div((R)1, base), mu2[m], e, q, a, bx);
      const R Iup = I[m];
      I[m] = fmar(e, Iup, fmar(q, Sp[m], a * (Sx[m] - Sp[m])));
      js = fmar(wm2[m], (double)I[m], js);
      if (PM) {  // App. A.2 for this ray: c_chi, c_eta (ingoing) or a_chi, a_eta (outgoing)
        const R rc = PL<R>::div((R)1, ch[m]);
        stage_put<KD>(tX + m * KD * kWave, k, lane,
                      (double)(-(Sx[m] * rc) * a + dz * (i2mu[m] * (e * (Sp[m] - Iup) - (Sp[m] - Sx[m]) * bx))));
        stage_put<KD>(tE + m * KD * kWave, k, lane, (double)(a * rc));
      }
      chp[m] = ch[m];
      Sp[m] = Sx[m];
    }
    return js;
  };

  // ---- sweep 1: ingoing rays (NMU + m), top -> bottom, I- = 0 at the top ----
  double chi0, eta0;
  vel_base(C, chunk, 0, fc, chi0, eta0);
  stg(xb + 2 * (size_t)f, chi0);
  stg(xb + 2 * (size_t)f + 1, eta0);
  vel_rays<NMU>(C, chunk, 0, fc, chi0, eta0, NMU, chp, Sp);
  stg(jm + f, 0.0);
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    I[m] = (R)0;
    if (PM) {  // ingoing rays at the top: I prescribed, no local dependence
      stage_put<KD>(tX + m * KD * kWave, 0, lane, 0.0);
      stage_put<KD>(tE + m * KD * kWave, 0, lane, 0.0);
    }
  }
  // Newton mode: the ingoing rays' derivatives leave KD depths at a time
  auto flush_down = [&](int k) {
    if (PM && (k % KD == KD - 1 || k == nz - 1)) {
#pragma unroll
      for (int m = 0; m < NMU; ++m) {
        stage_flush<KD>(tX + m * KD * kWave, C.DXR + (NMU + m) * rs, k - k % KD, nz, zp, f0, nnu, lane);
        stage_flush<KD>(tE + m * KD * kWave, C.DER + (NMU + m) * rs, k - k % KD, nz, zp, f0, nnu, lane);
      }
    }
  };
  flush_down(0);
  vel_rate_step<NMU>(C, chunk, 0, f, fc, NMU, I, wm2, true);
  for (int k = 1; k < nz; ++k) {
    vel_base(C, chunk, k, fc, chi0, eta0);
    const size_t kx = (size_t)k * fp + f;
    stg(xb + 2 * kx, chi0);
    stg(xb + 2 * kx + 1, eta0);
    vel_rays<NMU>(C, chunk, k, fc, chi0, eta0, NMU, ch, Sx);
    const double jac = step(k, (R)ldc(dzt + 2 * (k - 1)));  // segment k-1 -> k
    stg(jm + kx, jac);
    flush_down(k);
    vel_rate_step<NMU>(C, chunk, k, f, fc, NMU, I, wm2, true);
  }

  // Newton mode: the outgoing rays' derivatives leave KD depths at a time
  auto flush_up = [&](int k) {
    if (PM && k % KD == 0) {
#pragma unroll
      for (int m = 0; m < NMU; ++m) {
        stage_flush<KD>(tX + m * KD * kWave, C.DXR + m * rs, k, nz, zp, f0, nnu, lane);
        stage_flush<KD>(tE + m * KD * kWave, C.DER + m * rs, k, nz, zp, f0, nnu, lane);
      }
    }
  };
  // ---- sweep 2: outgoing rays (m), bottom -> top, I+ = B at the bottom ----
  {
    const int k = nz - 1;
    const size_t kx = (size_t)k * fp + f;
    vel_rays<NMU>(C, chunk, k, fc, ldg(xb + 2 * kx), ldg(xb + 2 * kx + 1), 0, chp, Sp);
    const R Bb = (R)ldg(C.Bnu + (size_t)k * nnu + fc);
    double jp = 0.0;
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      I[m] = Bb;
      jp = fmar(wm2[m], (double)Bb, jp);
      if (PM) {  // outgoing rays at the bottom: I prescribed
        stage_put<KD>(tX + m * KD * kWave, k, lane, 0.0);
        stage_put<KD>(tE + m * KD * kWave, k, lane, 0.0);
      }
    }
    vel_rate_step<NMU>(C, chunk, k, f, fc, 0, I, wm2, false);
    stage_put<KF>(tJ, k, lane, ldg(jm + kx) + jp);
    if (k % KF == 0) stage_flush<KF>(tJ, C.JT, k, nz, zp, f0, nnu, lane);
    flush_up(k);
  }
  for (int k = nz - 2; k >= 0; --k) {
    const size_t kx = (size_t)k * fp + f;
    vel_rays<NMU>(C, chunk, k, fc, ldg(xb + 2 * kx), ldg(xb + 2 * kx + 1), 0, ch, Sx);
    const double jp = step(k, (R)ldc(dzt + 2 * k));  // segment k -> k+1
    vel_rate_step<NMU>(C, chunk, k, f, fc, 0, I, wm2, false);
    stage_put<KF>(tJ, k, lane, ldg(jm + kx) + jp);
    if (k % KF == 0) stage_flush<KF>(tJ, C.JT, k, nz, zp, f0, nnu, lane);
    flush_up(k);
  }
}

template <typename R, bool PM, int NMU>
__global__ __launch_bounds__(256) void k_formal_vel(const ColDev* __restrict__ cols,
                                                    const Tile* __restrict__ tiles, int ntiles,
                                                    const Tile* __restrict__ mlist,
                                                    const int* __restrict__ mcount) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  Tile t;
  if (!pick_tile(tiles, ntiles, mlist, mcount, wave, t)) return;
  const int col = t.col, chunk = t.chunk;
  const ColDev& C = cols[col];
  if (uni(C.st->mode) != (PM ? kModeNewton : kModeF)) return;
  if (uni(C.st->cur_prec) != (sizeof(R) == sizeof(float) ? NLTE_FP32_FORM : NLTE_FP64)) return;
  extern __shared__ double stage[];  // [waves per block][VelStage doubles]
  formal_tile_vel<R, PM, NMU>(C, chunk, lane, stage + wave * VelStage<PM, NMU>::doubles);
}

template <typename R, bool PM>
static void launch_formal_vel_mode(int nmu, int wpb, hipStream_t s, const ColDev* cols,
                                   const Tile* tiles, int ntiles, const Tile* mlist,
                                   const int* mcount) {
  const int blocks = (ntiles + wpb - 1) / wpb;
  switch (nmu) {
#define NLTE_VEL_CASE(M)                                                                      \
  case M:                                                                                     \
    k_formal_vel<R, PM, M><<<blocks, 64 * wpb, (size_t)wpb * VelStage<PM, M>::doubles * 8, s>>>( \
        cols, tiles, ntiles, mlist, mcount);                                                  \
    break;
    NLTE_VEL_CASE(1) NLTE_VEL_CASE(2) NLTE_VEL_CASE(3) NLTE_VEL_CASE(4)
    NLTE_VEL_CASE(5) NLTE_VEL_CASE(6) NLTE_VEL_CASE(7) NLTE_VEL_CASE(8)
#undef NLTE_VEL_CASE
    default: break;
  }
}

void launch_formal_vel(bool fp32, bool newton, int nmu, int wpb, hipStream_t s, const ColDev* cols,
                       const Tile* tiles, int ntiles, const Tile* mlist, const int* mcount) {
  if (fp32) {
    if (newton)
      launch_formal_vel_mode<float, true>(nmu, wpb, s, cols, tiles, ntiles, mlist, mcount);
    else
      launch_formal_vel_mode<float, false>(nmu, wpb, s, cols, tiles, ntiles, mlist, mcount);
  } else {
    if (newton)
      launch_formal_vel_mode<double, true>(nmu, wpb, s, cols, tiles, ntiles, mlist, mcount);
    else
      launch_formal_vel_mode<double, false>(nmu, wpb, s, cols, tiles, ntiles, mlist, mcount);
  }
}

// Velocity fields: the same pair sums with the angle integral inside,
//   M1 = sum_nu cw_t sum_rays (w_m/2) A_t,ray V_t',ray D_chi,ray,
//   M2 = sum_nu cw_t sum_rays (w_m/2) A_t,ray g_t' V_t',ray (2 h nu^3/c^2 D_eta,ray - D_chi,ray),
// each ray with its own line profiles (depth-contiguous copies of the per-ray
// V tables) and local intensity derivatives (written depth-contiguous by the
// Newton-mode formal solution); the edges' cross-sections are the same for
// every ray.  One lane per depth, as pair_block.
__device__ void pair_vel(const ColDev& C, const PItem& it, int k) {
  const int nz = C.nz, L = C.L, zp = C.zp, nray = C.nray, nmu = C.nmu, nline = C.nline;
  const int f0 = it.f0, nf = it.f1 - it.f0, nt = it.nt, nu = it.nu;
  const size_t rs = (size_t)C.nnu * zp;
  const double *Vt[kPairBlk], *Vu[kPairBlk], *cw[kPairBlk];
  size_t rt[kPairBlk], ru[kPairBlk];  // ray steps (0: edge)
  int ft[kPairBlk], fu[kPairBlk];     // frequency steps (nz: line, 1: edge)
  double pa[kPairBlk], pb[kPairBlk], g0u[kPairBlk], gEu[kPairBlk];
  bool edge = false;
#pragma unroll
  for (int i = 0; i < kPairBlk; ++i) {
    const int t = it.t[i < nt ? i : 0];
    const TrDev& T = C.tr[t];
    const int wlo = uni(T.wlo), wl = uni(T.whi) - wlo;
    const double nl = C.eval_n[k * L + uni(T.lo)], nup = C.eval_n[k * L + uni(T.up)];
    if (t < nline) {
      Vt[i] = C.VRT + (size_t)nray * uni(T.voff) + (size_t)(f0 - wlo) * nz + k;
      rt[i] = (size_t)nz * wl;
      ft[i] = nz;
      pa[i] = nl - uni(T.g) * nup;
      pb[i] = 0.0;
    } else {
      Vt[i] = C.V + uni(T.voff) + (f0 - wlo);
      rt[i] = 0;
      ft[i] = 1;
      pa[i] = nl;
      pb[i] = C.rho_bf[k * C.nbf + (t - nline)] * nup;
      edge |= i < nt;
    }
    cw[i] = C.cw + uni(T.cwoff) + (f0 - wlo);
    const int u = it.u[i < nu ? i : 0];
    const TrDev& U = C.tr[u];
    const int ulo = uni(U.wlo), ul = uni(U.whi) - ulo;
    if (u < nline) {
      Vu[i] = C.VRT + (size_t)nray * uni(U.voff) + (size_t)(f0 - ulo) * nz + k;
      ru[i] = (size_t)nz * ul;
      fu[i] = nz;
      g0u[i] = uni(U.g);
      gEu[i] = 0.0;
    } else {
      Vu[i] = C.V + uni(U.voff) + (f0 - ulo);
      ru[i] = 0;
      fu[i] = 1;
      g0u[i] = 0.0;
      gEu[i] = C.rho_bf[k * C.nbf + (u - nline)];
      edge |= i < nu;
    }
  }
  const double* DX = C.DXR + (size_t)f0 * zp + k;
  const double* DE = C.DER + (size_t)f0 * zp + k;
  const double* EB = edge ? C.EbfT + (size_t)f0 * zp + k : DX;  // DX: any valid address
  double m1[kPairBlk][kPairBlk], m2[kPairBlk][kPairBlk];
#pragma unroll
  for (int i = 0; i < kPairBlk; ++i)
#pragma unroll
    for (int j = 0; j < kPairBlk; ++j) m1[i][j] = m2[i][j] = 0.0;
  for (int q = 0; q < nf; ++q) {
    const size_t oq = (size_t)q * zp;
    const double E = edge ? ldg(EB + oq) : 0.0;
    const double gam = ldc(C.gam + f0 + q);  // per-frequency: scalar load
    for (int r = 0; r < nray; ++r) {
      const double w = C.wm2[r < nmu ? r : r - nmu];
      const double dx = ldg(DX + r * rs + oq), de = ldg(DE + r * rs + oq);
      const double dd = gam * de - dx;
      double a[kPairBlk];
#pragma unroll
      for (int i = 0; i < kPairBlk; ++i)
        a[i] = i < nt ? w * ldc(cw[i] + q) * ldg(Vt[i] + r * rt[i] + (size_t)q * ft[i]) * (pa[i] - pb[i] * E) : 0.0;
#pragma unroll
      for (int j = 0; j < kPairBlk; ++j) {
        if (j >= nu) break;
        const double v = ldg(Vu[j] + r * ru[j] + (size_t)q * fu[j]);
        const double b = v * dx, c = (g0u[j] + gEu[j] * E) * v * dd;
#pragma unroll
        for (int i = 0; i < kPairBlk; ++i) {
          m1[i][j] = fma(a[i], b, m1[i][j]);
          m2[i][j] = fma(a[i], c, m2[i][j]);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kPairBlk; ++i)
#pragma unroll
    for (int j = 0; j < kPairBlk; ++j)
      if (i < nt && j < nu) {
        double* dst = C.M + ((size_t)(it.e0 + i * it.es + j) * nz + k) * 2;
        stg(dst, m1[i][j]);
        stg(dst + 1, m2[i][j]);
      }
}

// The same sums for a block whose transition lists hold at most one line
// each (lt, lu: its slot, or -1), taken in factored form: only a line's
// profile depends on the ray, so for each frequency the ray sums
//   D1 = sum_r w_r Dchi_r,       D2 = sum_r w_r Dd_r   (Dd = 2 h nu^3/c^2 Deta - Dchi),
//   X1 = sum_r w_r V_r Dchi_r,   X2 = sum_r w_r V_r Dd_r  (the list's line),
//   Z1 = sum_r w_r Vt_r Vu_r Dchi_r, Z2 likewise           (line with line)
// are formed once and every pair (t, u) of the block takes the one that
// fits it (edges enter with their ray-independent cross-sections), instead
// of every pair running its own sum over the rays.  Algebraically the sums
// of pair_vel; rounded in another order.
__device__ void pair_vel_one_line(const ColDev& C, const PItem& it, int k, int lt, int lu) {
  const int nz = C.nz, L = C.L, zp = C.zp, nray = C.nray, nmu = C.nmu, nline = C.nline;
  const int f0 = it.f0, nf = it.f1 - it.f0, nt = it.nt, nu = it.nu;
  const size_t rs = (size_t)C.nnu * zp;
  const double *At[kPairBlk], *Au[kPairBlk], *cw[kPairBlk];  // edges' cross-sections at f0
  double pa[kPairBlk], pb[kPairBlk], g0u[kPairBlk], gEu[kPairBlk];
  bool edge = false;
  const double *Vlt = nullptr, *Vlu = nullptr;  // the lines' per-ray V at f0, this depth
  size_t rlt = 0, rlu = 0;
#pragma unroll
  for (int i = 0; i < kPairBlk; ++i) {
    const int t = it.t[i < nt ? i : 0];
    const TrDev& T = C.tr[t];
    const int wlo = uni(T.wlo), wl = uni(T.whi) - wlo;
    const double nl = C.eval_n[k * L + uni(T.lo)], nup = C.eval_n[k * L + uni(T.up)];
    At[i] = C.V + uni(T.voff) + (f0 - wlo);  // (not read for the line)
    if (t < nline) {
      if (i == lt) {
        Vlt = C.VRT + (size_t)nray * uni(T.voff) + (size_t)(f0 - wlo) * nz + k;
        rlt = (size_t)nz * wl;
      }
      pa[i] = nl - uni(T.g) * nup;
      pb[i] = 0.0;
    } else {
      pa[i] = nl;
      pb[i] = C.rho_bf[k * C.nbf + (t - nline)] * nup;
      edge |= i < nt;
    }
    cw[i] = C.cw + uni(T.cwoff) + (f0 - wlo);
    const int u = it.u[i < nu ? i : 0];
    const TrDev& U = C.tr[u];
    const int ulo = uni(U.wlo), ul = uni(U.whi) - ulo;
    Au[i] = C.V + uni(U.voff) + (f0 - ulo);
    if (u < nline) {
      if (i == lu) {
        Vlu = C.VRT + (size_t)nray * uni(U.voff) + (size_t)(f0 - ulo) * nz + k;
        rlu = (size_t)nz * ul;
      }
      g0u[i] = uni(U.g);
      gEu[i] = 0.0;
    } else {
      g0u[i] = 0.0;
      gEu[i] = C.rho_bf[k * C.nbf + (u - nline)];
      edge |= i < nu;
    }
  }
  const bool same_line = lt >= 0 && lu >= 0 && it.t[lt] == it.u[lu];
  const double* DX = C.DXR + (size_t)f0 * zp + k;
  const double* DE = C.DER + (size_t)f0 * zp + k;
  const double* EB = edge ? C.EbfT + (size_t)f0 * zp + k : DX;  // DX: any valid address
  double m1[kPairBlk][kPairBlk], m2[kPairBlk][kPairBlk];
#pragma unroll
  for (int i = 0; i < kPairBlk; ++i)
#pragma unroll
    for (int j = 0; j < kPairBlk; ++j) m1[i][j] = m2[i][j] = 0.0;
  for (int q = 0; q < nf; ++q) {
    const size_t oq = (size_t)q * zp;
    const double E = edge ? ldg(EB + oq) : 0.0;
    const double gam = ldc(C.gam + f0 + q);  // per-frequency: scalar load
    double d1 = 0.0, d2 = 0.0, xt1 = 0.0, xt2 = 0.0, xu1 = 0.0, xu2 = 0.0, z1 = 0.0, z2 = 0.0;
    for (int r = 0; r < nray; ++r) {
      const double w = C.wm2[r < nmu ? r : r - nmu];
      const double dx = ldg(DX + r * rs + oq), de = ldg(DE + r * rs + oq);
      const double wx = w * dx, wd = w * (gam * de - dx);
      d1 += wx;
      d2 += wd;
      const double vt = lt >= 0 ? ldg(Vlt + r * rlt + (size_t)q * nz) : 0.0;
      const double vu = lu >= 0 ? (same_line ? vt : ldg(Vlu + r * rlu + (size_t)q * nz)) : 0.0;
      xt1 = fma(vt, wx, xt1);
      xt2 = fma(vt, wd, xt2);
      xu1 = fma(vu, wx, xu1);
      xu2 = fma(vu, wd, xu2);
      z1 = fma(vt * vu, wx, z1);
      z2 = fma(vt * vu, wd, z2);
    }
#pragma unroll
    for (int i = 0; i < kPairBlk; ++i) {
      if (i >= nt) break;
      const double a0 = ldc(cw[i] + q) * (pa[i] - pb[i] * E);
      const double at = i == lt ? 1.0 : ldc(At[i] + q);
#pragma unroll
      for (int j = 0; j < kPairBlk; ++j) {
        if (j >= nu) break;
        const double gu = g0u[j] + gEu[j] * E;
        const double au = j == lu ? 1.0 : ldc(Au[j] + q);
        double s1, s2;
        if (i == lt && j == lu) {
          s1 = z1;
          s2 = z2;
        } else if (i == lt) {
          s1 = au * xt1;
          s2 = au * xt2;
        } else if (j == lu) {
          s1 = at * xu1;
          s2 = at * xu2;
        } else {
          s1 = (at * au) * d1;
          s2 = (at * au) * d2;
        }
        m1[i][j] = fma(a0, s1, m1[i][j]);
        m2[i][j] = fma(a0 * gu, s2, m2[i][j]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kPairBlk; ++i)
#pragma unroll
    for (int j = 0; j < kPairBlk; ++j)
      if (i < nt && j < nu) {
        double* dst = C.M + ((size_t)(it.e0 + i * it.es + j) * nz + k) * 2;
        stg(dst, m1[i][j]);
        stg(dst + 1, m2[i][j]);
      }
}

// The pair-sum items of velocity-field columns, over the same work list (the
// other columns' items return at once): a kernel of its own, so that the ray
// loops do not cost the static kernel registers.
__global__ __launch_bounds__(64) void k_pairsum_vel(const ColDev* __restrict__ cols,
                                                    const int4* __restrict__ work, int nwork) {
  const int w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= nwork) return;
  const int4 wi = work[w];
  const ColDev& C = cols[uni(wi.x)];
  const int mode = ldc(&C.st->mode);
  if (!C.vel || mode != kModeNewton) return;
  const PItem it = ldc_rec(C.pitem + uni(wi.y));
  const int k = uni(wi.z) + threadIdx.x;
  if (k >= C.nz) return;
  // the line slots of the two lists (the factored form takes at most one each)
  int lt = -1, lu = -1, nlt = 0, nlu = 0;
  for (int i = 0; i < it.nt; ++i)
    if (it.t[i] < C.nline) {
      lt = i;
      ++nlt;
    }
  for (int j = 0; j < it.nu; ++j)
    if (it.u[j] < C.nline) {
      lu = j;
      ++nlu;
    }
  if (nlt <= 1 && nlu <= 1)
    pair_vel_one_line(C, it, k, lt, lu);
  else
    pair_vel(C, it, k);
}

void launch_pairsum_vel(const ColDev* cols, const int4* work, int nwork, hipStream_t s) {
  if (nwork > 0) k_pairsum_vel<<<nwork, 64, 0, s>>>(cols, work, nwork);
}

}  // namespace nlte
