// Tangent-linear Jacobian-vector products (Sect. 2.4.2, Eq. complex).
//
// The complex-step product Im F(n + i h v) / h of the paper is, for h far
// below the rounding level of the real part, the directional derivative
// dF/dn . v evaluated exactly: every O(h^2) term vanishes.  These kernels
// compute that derivative directly, carrying a derivative beside each
// quantity of Algorithm 1 (dual numbers) instead of complex arithmetic, so the
// work per depth point is one extra recurrence rather than a complex one:
//   opacity:  chi' and eta' are linear in v (the background and the lagged
//             scattering emissivity do not depend on n);  S' = (eta' - S chi')/chi
//   formal solution (Eqs. Iplus/Iminus, App. A.1): for each segment with
//             optical depth x, x' = dz (chi'_k + chi'_k+1) / (2 mu), and
//             e' = -e x',  a' = (b/x) x',  b' = (e - b/x) x', so that
//             I'_k = I'_prev e + I_prev e' + a' S_k + a S'_k + b' S_prev + b S'_prev
//             with I' = 0 at both boundaries;  J' = sum_m w_m/2 (I+' + I-')
//   rates:    R_lu' and the J part of R_ul' over J' (Eqs. Rij, Rji)
//   assembly: F'_i = sum_t +-(v_l Rtot_lu + n_l R_lu' - v_u Rtot_ul - n_u R_ul'),
//             and -sum_l v_l on the conservation rows (Eqs. residuals_1/2).
// Everything runs in FP64 whatever the column's formal-solution precision.
//
// Inputs per column: the populations n in ColDev::n, the direction v in
// ColDev::eval_n, the total rates of n in ColDev::Rtot and the conservation
// rows in ColDev::rows_frozen (both from an evaluation at n), the lagged J.
// Output: J v in ColDev::F.  Scratch: XS (chi, S), Dchi (chi'), Deta (S'),
// Jm (J'), RJ (R').  Three launches: the formal solution (which makes the
// opacity on its way down), the rate derivatives, the assembly.  A column
// takes part when its state has tan_pending set (its mode is then idle, so
// the residual kernels skip it).  Columns with a velocity field run their
// own formal-solution variant (k_tan_formal_vel) and keep the angle integral
// inside the line rates' frequency sum.
#include "nlte_internal.h"

namespace nlte {

namespace {

constexpr int kTanRateSplit = 8;   // blocks per column (rate derivatives)
constexpr int kTanRateThreads = 256;

__device__ __forceinline__ bool tan_on(const ColDev& C) {
  return __builtin_amdgcn_readfirstlane(C.st->tan_pending) != 0;
}

// e = exp(-x) and the piecewise-linear coefficients a = 1 - (1 - e)/x,
// b = (1 - e)/x - e of App. A.1, with bx = b / x (the derivative of a).
// Below x = 0.1 the three come from their Taylor series about 0,
//   a  = sum_{m>=1} (-1)^(m+1) x^m / (m+1)!,
//   b  = sum_{m>=1} (-1)^(m+1) m x^m / (m+1)!,
//   bx = sum_{m>=1} (-1)^(m+1) m x^(m-1) / (m+1)!,
// ten terms (truncation below 1e-17 relative there); above, 1 - e has no
// cancellation (it is at least 0.095) and rx = 1/x (shared by the angles of
// a segment, passed in) serves both quotients.
__device__ __forceinline__ void seg_ab(double x, double rx, double& e, double& a, double& b,
                                       double& bx) {
  e = exp(-x);
  if (x < 0.1) {
    constexpr int kTerms = 10;
    double fa = 0.0, fb = 0.0;
    double fact = 1.0;  // (m+1)! for m = kTerms
    for (int j = 2; j <= kTerms + 1; ++j) fact *= j;
#pragma unroll
    for (int m = kTerms; m >= 1; --m) {
      const double c = ((m & 1) ? 1.0 : -1.0) / fact;  // (-1)^(m+1) / (m+1)!
      fa = fma(fa, x, c);
      fb = fma(fb, x, c * m);
      fact /= (m + 1);
    }
    // fa = sum c_m x^(m-1), fb = sum c_m m x^(m-1)
    a = fa * x;
    bx = fb;
    b = fb * x;
  } else {
    const double t1 = (1.0 - e) * rx;
    a = 1.0 - t1;
    b = t1 - e;
    bx = b * rx;
  }
}

// chi, S, chi' = d chi . v and S' at depth k and frequency f (f < nnu) of
// a chunk; the transition lists of the chunk are the same for every lane.
__device__ __forceinline__ void tan_opacity(const ColDev& C, int chunk, int k, int f, int L,
                                            int nnu, int nbf, int nline, double gam,
                                            double& X, double& S, double& Xd, double& Sd) {
  const double* nk = C.n + (size_t)k * L;
  const double* vk = C.eval_n + (size_t)k * L;
  double chi = 0.0, et = 0.0, chid = 0.0, etd = 0.0;
  // the chunk's transition lists, their windows and the depth's level
  // populations are the same for every lane: scalar loads (ldc), which do
  // not wait for the wave's vector loads and stores in flight
  const int l0 = ldc(C.ch_lptr + chunk), l1 = ldc(C.ch_lptr + chunk + 1);
  for (int j = l0; j < l1; ++j) {
    const TrDev* T = C.tr + ldc(C.ch_line + j);
    const int wlo = ldc(&T->wlo), wl = ldc(&T->whi) - wlo, q = f - wlo;
    const double g = ldc(&T->g), nu = ldc(nk + ldc(&T->up)), vu = ldc(vk + ldc(&T->up));
    const double nl = ldc(nk + ldc(&T->lo)), vl = ldc(vk + ldc(&T->lo));
    if (q < 0 || q >= wl) continue;
    const double V = C.V[ldc(&T->voff) + (size_t)k * wl + q];
    const double c1 = g * nu, c1d = g * vu;
    chi += V * (nl - c1);
    et += V * c1;
    chid += V * (vl - c1d);
    etd += V * c1d;
  }
  double A1 = 0.0, A2 = 0.0, A1d = 0.0, A2d = 0.0;
  const int e0 = ldc(C.ch_eptr + chunk), e1 = ldc(C.ch_eptr + chunk + 1);
  for (int j = e0; j < e1; ++j) {
    const int t = ldc(C.ch_edge + j);
    const TrDev* T = C.tr + t;
    const int wlo = ldc(&T->wlo), q = f - wlo;
    const double rb = ldc(C.rho_bf + (size_t)k * nbf + (t - nline));
    const double nl = ldc(nk + ldc(&T->lo)), vl = ldc(vk + ldc(&T->lo));
    const double nc = ldc(nk + L - 1), vc = ldc(vk + L - 1);
    if (q < 0 || q >= ldc(&T->whi) - wlo) continue;
    const double al = C.V[ldc(&T->voff) + q];
    A1 += al * nl;
    A2 += al * rb * nc;
    A1d += al * vl;
    A2d += al * rb * vc;
  }
  const size_t kf = (size_t)k * nnu + f;
  const double E = nbf ? C.Ebf[kf] : 0.0;
  X = (C.chi_c[k] + C.chi_sca[k]) + chi + (A1 - E * A2);
  double eta = (C.bg_eta ? 1.0 : C.chi_c[k]) * C.EC[kf] + gam * (et + E * A2);
  if (C.has_sca) eta += C.chi_sca[k] * C.Jdag[kf];
  Xd = chid + (A1d - E * A2d);
  const double etad = gam * (etd + E * A2d);
  const double rX = 1.0 / X;
  S = eta * rX;
  Sd = (etad - S * Xd) * rX;
}

// One segment of every ray of a lane (NMU angles in registers): I and I'
// advance from the segment's start (S0, S0') to its end (S1, S1');
// returns sum_m w_m/2 I'_m at the end.  x_m = sx / (2 mu_m), so one
// reciprocal of sx gives every 1/x_m = (2 mu_m) / sx.
template <int NMU>
__device__ __forceinline__ double tan_segment(double sx, double sxd, double S0, double Sd0,
                                              double S1, double Sd1, const double (&i2mu)[kMaxMu],
                                              const double (&mu2)[kMaxMu],
                                              const double (&wm2)[kMaxMu], double (&I)[kMaxMu],
                                              double (&Id)[kMaxMu]) {
  double jd = 0.0;
  const double rs = 1.0 / sx;
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    const double x = sx * i2mu[m], xd = sxd * i2mu[m];
    double e, a, b, bx;
    seg_ab(x, rs * mu2[m], e, a, b, bx);
    const double ed = -e * xd, ad = bx * xd, bd = (e - bx) * xd;
    const double In = I[m] * e + a * S1 + b * S0;
    const double Idn = Id[m] * e + I[m] * ed + ad * S1 + a * Sd1 + bd * S0 + b * Sd0;
    I[m] = In;
    Id[m] = Idn;
    jd += wm2[m] * Idn;
  }
  return jd;
}

// Intensities and their derivatives along every ray of one frequency (one
// lane per frequency of a chunk), all angles at once.  The downward sweep
// makes chi, S and their derivatives depth by depth and parks them for the
// upward one; J' of each depth goes to Jm (the ingoing part on the way down,
// the outgoing part added on the way up by the same lane).
template <int NMU>
__global__ __launch_bounds__(64) void k_tan_formal(const ColDev* __restrict__ cols,
                                                   const Tile* __restrict__ tiles, int ntiles) {
  if ((int)blockIdx.x >= ntiles) return;
  const ColDev& C = cols[uni(tiles[blockIdx.x].col)];
  if (!tan_on(C)) return;
  if (uni(C.nmu) != NMU) return;
  const int chunk = uni(tiles[blockIdx.x].chunk);
  const int nz = C.nz, nnu = C.nnu, fp = C.fp, L = C.L, nbf = C.nbf, nline = C.nline;
  const int f = chunk * kWave + (int)threadIdx.x;
  if (f >= nnu) return;
  double* __restrict__ XS = C.XS;
  double* __restrict__ Dx = C.Dchi;
  double* __restrict__ Ds = C.Deta;
  double* __restrict__ Jd = C.Jm;
  const double* __restrict__ dzs = C.dz;
  const double gam = C.gam[f];
  double i2mu[kMaxMu], mu2[kMaxMu], wm2[kMaxMu];
#pragma unroll
  for (int m = 0; m < kMaxMu; ++m) {
    i2mu[m] = C.inv2mu[m];
    mu2[m] = m < NMU ? 1.0 / i2mu[m] : 0.0;
    wm2[m] = C.wm2[m];
  }
  double I[kMaxMu], Id[kMaxMu];
  // ingoing rays, top -> bottom (I- = 0 at the top)
#pragma unroll
  for (int m = 0; m < kMaxMu; ++m) I[m] = Id[m] = 0.0;
  double X0, S0, Xd0, Sd0;
  tan_opacity(C, chunk, 0, f, L, nnu, nbf, nline, gam, X0, S0, Xd0, Sd0);
  size_t kx = (size_t)f;
  XS[2 * kx] = X0;
  XS[2 * kx + 1] = S0;
  Dx[kx] = Xd0;
  Ds[kx] = Sd0;
  Jd[kx] = 0.0;
  for (int k = 1; k < nz; ++k) {
    double X1, S1, Xd1, Sd1;
    tan_opacity(C, chunk, k, f, L, nnu, nbf, nline, gam, X1, S1, Xd1, Sd1);
    kx = (size_t)k * fp + f;
    XS[2 * kx] = X1;
    XS[2 * kx + 1] = S1;
    Dx[kx] = Xd1;
    Ds[kx] = Sd1;
    const double dz = dzs[k - 1];
    Jd[kx] = tan_segment<NMU>(dz * (X0 + X1), dz * (Xd0 + Xd1), S0, Sd0, S1, Sd1, i2mu, mu2, wm2, I, Id);
    X0 = X1; S0 = S1; Xd0 = Xd1; Sd0 = Sd1;
  }
  // outgoing rays, bottom -> top (I+ = B at the bottom, I+' = 0)
  const double Bb = C.Bnu[(size_t)(nz - 1) * nnu + f];
#pragma unroll
  for (int m = 0; m < kMaxMu; ++m) {
    I[m] = Bb;
    Id[m] = 0.0;
  }
  for (int k = nz - 2; k >= 0; --k) {
    kx = (size_t)k * fp + f;
    const double X1 = XS[2 * kx], S1 = XS[2 * kx + 1], Xd1 = Dx[kx], Sd1 = Ds[kx];
    const double dz = dzs[k];
    Jd[kx] += tan_segment<NMU>(dz * (X0 + X1), dz * (Xd0 + Xd1), S0, Sd0, S1, Sd1, i2mu, mu2, wm2, I, Id);
    X0 = X1; S0 = S1; Xd0 = Xd1; Sd0 = Sd1;
  }
}

// Velocity fields (Sect. 3.5): every ray has its own line opacity, so each
// carries its own chi, S and derivatives through the recursion (segment
// optical depths differ between rays); the ray-independent part (background,
// edges) is made once per depth on the way down and parked.  Each ray's I'
// is kept ([ray][k][fp] in the column's per-ray derivative buffer, free while
// a tangent product runs) for the line rates, whose angle integral stays
// inside the frequency sum.

// Ray-independent chi, eta and derivatives at (k, f): background, edges and
// the lagged scattering emissivity.
__device__ __forceinline__ void tan_base_vel(const ColDev& C, int chunk, int k, int f, int L, int nnu,
                                             int nbf, int nline, double gam, double& X, double& Et,
                                             double& Xd, double& Ed) {
  const double* nk = C.n + (size_t)k * L;
  const double* vk = C.eval_n + (size_t)k * L;
  double A1 = 0.0, A2 = 0.0, A1d = 0.0, A2d = 0.0;
  const int e0 = ldc(C.ch_eptr + chunk), e1 = ldc(C.ch_eptr + chunk + 1);
  for (int j = e0; j < e1; ++j) {
    const int t = ldc(C.ch_edge + j);
    const TrDev* T = C.tr + t;
    const int wlo = ldc(&T->wlo), q = f - wlo;
    const double rb = ldc(C.rho_bf + (size_t)k * nbf + (t - nline));
    const double nl = ldc(nk + ldc(&T->lo)), vl = ldc(vk + ldc(&T->lo));
    const double nc = ldc(nk + L - 1), vc = ldc(vk + L - 1);
    if (q < 0 || q >= ldc(&T->whi) - wlo) continue;
    const double al = C.V[ldc(&T->voff) + q];
    A1 += al * nl;
    A2 += al * rb * nc;
    A1d += al * vl;
    A2d += al * rb * vc;
  }
  const size_t kf = (size_t)k * nnu + f;
  const double E = nbf ? C.Ebf[kf] : 0.0;
  X = (C.chi_c[k] + C.chi_sca[k]) + (A1 - E * A2);
  Et = (C.bg_eta ? 1.0 : C.chi_c[k]) * C.EC[kf] + gam * (E * A2);
  if (C.has_sca) Et += C.chi_sca[k] * C.Jdag[kf];
  Xd = A1d - E * A2d;
  Ed = gam * (E * A2d);
}

// chi, S and their derivatives at (k, f) of the rays r0 .. r0 + NMU - 1.
template <int NMU>
__device__ __forceinline__ void tan_rays_vel(const ColDev& C, int chunk, int k, int f, int L, int r0,
                                             double gam, double X0, double E0, double Xd0, double Ed0,
                                             double (&X)[NMU], double (&S)[NMU], double (&Xd)[NMU],
                                             double (&Sd)[NMU]) {
  const double* nk = C.n + (size_t)k * L;
  const double* vk = C.eval_n + (size_t)k * L;
  double et[NMU], etd[NMU];
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    X[m] = X0;
    Xd[m] = Xd0;
    et[m] = 0.0;
    etd[m] = 0.0;
  }
  const int nz = C.nz;
  const int l0 = ldc(C.ch_lptr + chunk), l1 = ldc(C.ch_lptr + chunk + 1);
  for (int j = l0; j < l1; ++j) {
    const TrDev* T = C.tr + ldc(C.ch_line + j);
    const int wlo = ldc(&T->wlo), wl = ldc(&T->whi) - wlo, q = f - wlo;
    const double g = ldc(&T->g), nu = ldc(nk + ldc(&T->up)), vu = ldc(vk + ldc(&T->up));
    const double nl = ldc(nk + ldc(&T->lo)), vl = ldc(vk + ldc(&T->lo));
    const size_t voff = ldc(&T->voff);
    if (q < 0 || q >= wl) continue;
    const double c1 = g * nu, c1d = g * vu;
    const double c0 = nl - c1, c0d = vl - c1d;
    const double* vr = C.VR + (size_t)C.nray * voff + ((size_t)r0 * nz + k) * wl + q;
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      const double V = vr[(size_t)m * nz * wl];
      X[m] += V * c0;
      Xd[m] += V * c0d;
      et[m] += V * c1;
      etd[m] += V * c1d;
    }
  }
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    const double rX = 1.0 / X[m];
    S[m] = (E0 + gam * et[m]) * rX;
    Sd[m] = ((Ed0 + gam * etd[m]) - S[m] * Xd[m]) * rX;
  }
}

template <int NMU>
__global__ __launch_bounds__(64) void k_tan_formal_vel(const ColDev* __restrict__ cols,
                                                       const Tile* __restrict__ tiles, int ntiles) {
  if ((int)blockIdx.x >= ntiles) return;
  const ColDev& C = cols[uni(tiles[blockIdx.x].col)];
  if (!tan_on(C)) return;
  if (uni(C.nmu) != NMU) return;
  const int chunk = uni(tiles[blockIdx.x].chunk);
  const int nz = C.nz, nnu = C.nnu, fp = C.fp, L = C.L, nbf = C.nbf, nline = C.nline;
  const int f = chunk * kWave + (int)threadIdx.x;
  if (f >= nnu) return;
  double* __restrict__ XS = C.XS;    // ray-independent chi, eta
  double* __restrict__ Dx = C.Dchi;  // and their derivatives
  double* __restrict__ De = C.Deta;
  double* __restrict__ Jd = C.Jm;
  double* __restrict__ Id_out = C.DXR;  // [ray][k][fp] I' of every ray
  const size_t rs = (size_t)nz * fp;
  const double* __restrict__ dzs = C.dz;
  const double gam = C.gam[f];
  double i2mu[NMU], wm2[NMU];
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    i2mu[m] = C.inv2mu[m];
    wm2[m] = C.wm2[m];
  }
  double I[NMU], Id[NMU], Xp[NMU], Sp[NMU], Xdp[NMU], Sdp[NMU];
  double X[NMU], S[NMU], Xd[NMU], Sd[NMU];
  // one segment of every ray of the sweep, from (Xp, Sp) to (X, S)
  auto step = [&](double dz, int k, int r0) {
    double jd = 0.0;
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      const double sx = dz * (Xp[m] + X[m]), sxd = dz * (Xdp[m] + Xd[m]);
      const double x = sx * i2mu[m], xd = sxd * i2mu[m];
      double e, a, b, bx;
      seg_ab(x, 1.0 / x, e, a, b, bx);
      const double ed = -e * xd, ad = bx * xd, bd = (e - bx) * xd;
      const double In = I[m] * e + a * S[m] + b * Sp[m];
      const double Idn = Id[m] * e + I[m] * ed + ad * S[m] + a * Sd[m] + bd * Sp[m] + b * Sdp[m];
      I[m] = In;
      Id[m] = Idn;
      jd += wm2[m] * Idn;
      Id_out[(size_t)(r0 + m) * rs + (size_t)k * fp + f] = Idn;
      Xp[m] = X[m];
      Sp[m] = S[m];
      Xdp[m] = Xd[m];
      Sdp[m] = Sd[m];
    }
    return jd;
  };
  // ingoing rays (NMU + m), top -> bottom (I- = 0 at the top)
  double X0, E0, Xd0, Ed0;
  tan_base_vel(C, chunk, 0, f, L, nnu, nbf, nline, gam, X0, E0, Xd0, Ed0);
  size_t kx = (size_t)f;
  XS[2 * kx] = X0;
  XS[2 * kx + 1] = E0;
  Dx[kx] = Xd0;
  De[kx] = Ed0;
  Jd[kx] = 0.0;
  tan_rays_vel<NMU>(C, chunk, 0, f, L, NMU, gam, X0, E0, Xd0, Ed0, Xp, Sp, Xdp, Sdp);
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    I[m] = Id[m] = 0.0;
    Id_out[(size_t)(NMU + m) * rs + f] = 0.0;
  }
  for (int k = 1; k < nz; ++k) {
    tan_base_vel(C, chunk, k, f, L, nnu, nbf, nline, gam, X0, E0, Xd0, Ed0);
    kx = (size_t)k * fp + f;
    XS[2 * kx] = X0;
    XS[2 * kx + 1] = E0;
    Dx[kx] = Xd0;
    De[kx] = Ed0;
    tan_rays_vel<NMU>(C, chunk, k, f, L, NMU, gam, X0, E0, Xd0, Ed0, X, S, Xd, Sd);
    Jd[kx] = step(dzs[k - 1], k, NMU);
  }
  // outgoing rays (m), bottom -> top (I+ = B at the bottom, I+' = 0)
  {
    const int k = nz - 1;
    kx = (size_t)k * fp + f;
    tan_rays_vel<NMU>(C, chunk, k, f, L, 0, gam, XS[2 * kx], XS[2 * kx + 1], Dx[kx], De[kx], Xp, Sp,
                      Xdp, Sdp);
    const double Bb = C.Bnu[(size_t)k * nnu + f];
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      I[m] = Bb;
      Id[m] = 0.0;
      Id_out[(size_t)m * rs + kx] = 0.0;
    }
  }
  for (int k = nz - 2; k >= 0; --k) {
    kx = (size_t)k * fp + f;
    tan_rays_vel<NMU>(C, chunk, k, f, L, 0, gam, XS[2 * kx], XS[2 * kx + 1], Dx[kx], De[kx], X, S, Xd,
                      Sd);
    Jd[kx] += step(dzs[k], k, 0);
  }
}

// R_lu' and R_ul' of every (depth, transition): one wave per pair, lanes
// strided over the transition's window, then a wave reduction.  Stored in RJ
// as [nz][ntr][2] (rows of nrseg >= ntr entries).
__global__ __launch_bounds__(kTanRateThreads) void k_tan_rates(const ColDev* __restrict__ cols,
                                                               const int* __restrict__ act) {
  const int ci = blockIdx.x / kTanRateSplit, part = blockIdx.x - ci * kTanRateSplit;
  const ColDev& C = cols[act ? act[ci] : ci];
  if (!tan_on(C)) return;
  const int nz = C.nz, ntr = C.ntr, nline = C.nline, nnu = C.nnu, fp = C.fp;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int kWaves = kTanRateThreads / 64;
  for (int it = part * kWaves + wave; it < nz * ntr; it += kTanRateSplit * kWaves) {
    const int k = it / ntr, t = it - k * ntr;
    const TrDev& T = C.tr[t];
    const int wlo = T.wlo, wl = T.whi - T.wlo;
    const double* cw = C.cw + T.cwoff;
    const double* Jk = C.Jm + (size_t)k * fp + wlo;
    double s1 = 0.0, s2 = 0.0;
    if (t < nline && C.vel) {
      // velocity fields: the angle integral inside, sum_rays (w_m/2) V_ray I'_ray
      const int nray = C.nray, nmu = C.nmu;
      const size_t vs = (size_t)nz * wl, rs = (size_t)nz * fp;
      const double* V = C.VR + (size_t)nray * T.voff + (size_t)k * wl;
      const double* Ik = C.DXR + (size_t)k * fp + wlo;
      for (int q = lane; q < wl; q += kWave) {
        double u = 0.0;
        for (int r = 0; r < nray; ++r) u += C.wm2[r < nmu ? r : r - nmu] * V[r * vs + q] * Ik[r * rs + q];
        s1 += cw[q] * u;
      }
    } else if (t < nline) {
      const double* V = C.V + T.voff + (size_t)k * wl;
      for (int q = lane; q < wl; q += kWave) s1 += cw[q] * V[q] * Jk[q];
    } else {
      const double* al = C.V + T.voff;
      const double* E = C.Ebf + (size_t)k * nnu + wlo;
      for (int q = lane; q < wl; q += kWave) {
        const double x = cw[q] * al[q] * Jk[q];
        s1 += x;
        s2 += x * E[q];
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      s1 += __shfl_xor(s1, o);
      s2 += __shfl_xor(s2, o);
    }
    if (lane == 0) {
      const double Rul = t < nline ? T.g * s1 : C.rho_bf[(size_t)k * C.nbf + (t - nline)] * s2;
      double* out = C.RJ + ((size_t)k * C.nrseg + t) * 2;
      out[0] = s1;
      out[1] = Rul;
    }
  }
}

// F' of one depth per thread (the rows of a thread live in its own LDS row).
constexpr int kTanAsmDepths = 64;
__global__ __launch_bounds__(kTanAsmDepths) void k_tan_assemble(const ColDev* __restrict__ cols,
                                                                const int* __restrict__ act,
                                                                int nsub) {
  __shared__ double sF[kTanAsmDepths][kMaxLev + 1];
  const int ci = blockIdx.x / nsub, sub = blockIdx.x - ci * nsub;
  const ColDev& C = cols[act ? act[ci] : ci];
  if (!tan_on(C)) return;
  const int nz = C.nz, L = C.L, ntr = C.ntr;
  const int k = sub * kTanAsmDepths + (int)threadIdx.x;
  if (k >= nz) return;
  double* Fk = sF[threadIdx.x];
  const double* nk = C.n + (size_t)k * L;
  const double* vk = C.eval_n + (size_t)k * L;
  for (int i = 0; i < L; ++i) Fk[i] = 0.0;
  const double* Rd = C.RJ + (size_t)k * C.nrseg * 2;
  const double* Rt = C.Rtot + (size_t)k * ntr * 2;
  for (int t = 0; t < ntr; ++t) {
    const TrDev& T = C.tr[t];
    const int lo = T.lo, up = T.up;
    const double kap = (vk[lo] * Rt[2 * t] + nk[lo] * Rd[2 * t]) -
                       (vk[up] * Rt[2 * t + 1] + nk[up] * Rd[2 * t + 1]);
    Fk[lo] += kap;
    Fk[up] -= kap;
  }
  double sum = 0.0;
  for (int i = 0; i < L; ++i) sum += vk[i];
  Fk[C.rows_frozen[k]] = -sum;
  for (int i = 0; i < L; ++i) C.F[(size_t)k * L + i] = Fk[i];
}

}  // namespace

hipError_t launch_tangent(const BatchWork& bw, hipStream_t s) {
  if (bw.ntiles <= 0) return hipSuccess;
  const int nblk = bw.act ? bw.nact : bw.ncol;
  // one instantiation per angle count present (tile groups are per angle
  // count; each launch covers the tiles of its groups)
  for (int g = 0; g < bw.ngroup; ++g) {
    const TileGroup& G = bw.groups[g];
    const Tile* tl = bw.tiles + G.first;
    if (G.vel) {
      switch (G.nmu) {
#define TFV(M) \
  case M: k_tan_formal_vel<M><<<G.count, 64, 0, s>>>(bw.cols, tl, G.count); break;
        TFV(1) TFV(2) TFV(3) TFV(4) TFV(5) TFV(6) TFV(7) TFV(8)
#undef TFV
        default: return hipErrorInvalidValue;
      }
      continue;
    }
    switch (G.nmu) {
#define TF(M) \
  case M: k_tan_formal<M><<<G.count, 64, 0, s>>>(bw.cols, tl, G.count); break;
      TF(1) TF(2) TF(3) TF(4) TF(5) TF(6) TF(7) TF(8)
#undef TF
      default: return hipErrorInvalidValue;
    }
  }
  k_tan_rates<<<nblk * kTanRateSplit, kTanRateThreads, 0, s>>>(bw.cols, bw.act);
  const int nsub = (bw.maxnz + kTanAsmDepths - 1) / kTanAsmDepths;
  k_tan_assemble<<<nblk * nsub, kTanAsmDepths, 0, s>>>(bw.cols, bw.act, nsub);
  return hipGetLastError();
}

}  // namespace nlte
