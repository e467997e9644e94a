// Residual F(n) on the device (Algorithm 1): opacity and emissivity assembly
// (Eqs. chi, eta), the short-characteristics formal solution for every
// frequency and ray (Eqs. Iplus, Iminus, App. A.1), the angle quadrature into
// the mean intensity, the frequency quadrature into radiative rates
// (Eqs. Rij, Rji), the rate-equation residual with conservation rows
// (Eqs. residuals_1, residuals_2) and, in Newton mode, the block-Jacobi
// preconditioner (Sect. 2.5.2 first solution, App. A.2).
//
// Work decomposition (one launch of each per residual call of a batch):
//   k_coef    : one block per column; the level coefficients of the
//               evaluation, transition-major, so that one scalar load brings
//               a transition's values for several depths.
//   k_opacity : chi and S of a 64-frequency chunk, a few depths per wave;
//               launches over few chunks spread a chunk's depth groups over
//               waves.  Large FP32 launches skip it: the first sweep of
//               k_formal makes the same opacity itself.
//   k_formal  : one wavefront per chunk of 64 consecutive frequencies of one
//               column, one lane per frequency carrying all 2 x nmu rays
//               through the depth recursion in registers.  The first sweep
//               runs top -> bottom (ingoing rays) and parks their share of J
//               in a [k][nu] scratch row; the second runs bottom -> top
//               (outgoing rays) and writes J.  In Newton mode it also writes
//               the angle-averaged local intensity derivatives.
//   k_formal_scan: the same for columns created with NLTE_DEPTH_SCAN, as
//               parallel scans of affine maps over depth (one workgroup per
//               frequency, one thread per depth).
//   k_depthwork: one lane per depth, one wavefront per (column, block of a
//               piece, 64 depths): rate integrals summed in frequency order
//               (no cross-lane reductions, independent of batching), and in
//               Newton mode the preconditioner pair sums, per (column, piece
//               of constant transition set, block of pairs, 64 depths).
//   k_assemble: rates, rate-equation residual, conservation rows, scaled
//               residual per depth; one block per (column, 16 depths).
//   k_pblock  : Newton mode; the preconditioner blocks from the total rates
//               and the pair sums.
// Columns with a velocity field run their own formal-solution and pair-sum
// kernels (nlte_velocity.hip); the other launches are shared.
#include <type_traits>

#include "nlte_kernels.h"

namespace nlte {

// ---------------------------------------------------------------------------
// opacity and emissivity, Eqs. chi and eta
// ---------------------------------------------------------------------------
// Per evaluation, k_coef turns the populations into two FP64 numbers per
// transition and depth, stored transition-major ([ntr + 2][nz][2]):
//   lines: c0 = n_l - g n_u, c1 = g n_u;   edges: c0 = n_l, c1 = (n*_l/n*_c) n_c;
//   row ntr: chi_c + chi_sca, chi_c (1 when the caller gave eta_c);
//   row ntr + 1: chi_sca, dz,
// so that for every (k, nu), with E = exp(-h nu / kT) and EC the background
// emission table (B_nu, or eta_c),
//   chi = chi_c + chi_sca + sum_lines V c0 + sum_edges alpha (c0 - E c1)
//   eta = c1(ntr) EC + chi_sca J' + (2 h nu^3/c^2) (sum_lines V c1 + E sum_edges alpha c1).
// In the FP32 form, B_nu and E are made in FP32 from T and nu where they are
// used (one exponential per (k, nu), shared by the rays), unless the caller
// gave the background emissivity; the FP64 form reads its FP64 tables.
//
// With per-step mode lists (ml.mlist non-NULL), each column of a listed group
// also appends its chunks to the list of the formal-solution launch that
// will evaluate it (one atomic per column; the order within a list depends
// on the atomics, which only moves waves between CUs: each tile is evaluated
// by one wave wherever it runs, so the results are the same bits).
struct ModeLists {
  const int* gidx;
  Tile* mlist;
  int* mcount;
  int ntiles;
  int first[kMaxGroups];  // a group's first tile
  int fp32[kMaxGroups];   // FP32-form group: fallback columns go to lists 2, 3
};

__global__ __launch_bounds__(256) void k_coef(const ColDev* __restrict__ cols,
                                              const int* __restrict__ act, ModeLists ml) {
  const int c = act ? act[blockIdx.x] : blockIdx.x;
  const ColDev& C = cols[c];
  const int mode = uni(C.st->mode);
  if (mode == kModeIdle) return;
  if (ml.mlist) {
    const int g = ml.gidx[c];
    if (g >= 0) {
      __shared__ int base;
      const int li = (mode == kModeNewton ? 1 : 0) +
                     (ml.fp32[g] && uni(C.st->cur_prec) == NLTE_FP64 ? 2 : 0);
      const int nch = C.nchunk;
      if (threadIdx.x == 0) base = atomicAdd(ml.mcount + 4 * g + li, nch);
      __syncthreads();
      Tile* dst = ml.mlist + (size_t)li * ml.ntiles + ml.first[g] + base;
      for (int ch = threadIdx.x; ch < nch; ch += blockDim.x) dst[ch] = Tile{c, ch};
    }
  }
  const int nz = C.nz, ntr = C.ntr, nline = C.nline, L = C.L;
  const int per = ntr + 2;
  for (int id = threadIdx.x; id < nz * per; id += blockDim.x) {
    const int t = id / nz, k = id - t * nz;
    const double* nk = C.eval_n + k * L;
    double c0, c1;
    if (t < nline) {
      const TrDev& T = C.tr[t];
      c1 = T.g * nk[T.up];
      c0 = nk[T.lo] - c1;
    } else if (t < ntr) {
      c0 = nk[C.tr[t].lo];
      c1 = C.rho_bf[k * C.nbf + (t - nline)] * nk[L - 1];
    } else if (t == ntr) {
      c0 = C.chi_c[k] + C.chi_sca[k];
      c1 = C.bg_eta ? 1.0 : C.chi_c[k];
    } else {
      c0 = C.chi_sca[k];
      c1 = k + 1 < nz ? C.dz[k] : 0.0;
    }
    const size_t o = 2 * (size_t)id;
    ((double*)C.coef)[o] = c0;
    ((double*)C.coef)[o + 1] = c1;
  }
}

// Tables and angle constants in the precision of the depth recursion.
template <typename R> struct FTab;
template <> struct FTab<double> {
  static __device__ __forceinline__ const double* V(const ColDev& C) { return C.V; }
  static __device__ __forceinline__ const double* B(const ColDev& C) { return C.EC; }
  static __device__ __forceinline__ const double* E(const ColDev& C) { return C.Ebf; }
  static __device__ __forceinline__ double wm2(const ColDev& C, int m) { return C.wm2[m]; }
  static __device__ __forceinline__ double i2mu(const ColDev& C, int m) { return C.inv2mu[m]; }
};
template <> struct FTab<float> {
  static __device__ __forceinline__ const float* V(const ColDev& C) { return C.Vf; }
  static __device__ __forceinline__ const float* B(const ColDev& C) { return C.ECf; }
  static __device__ __forceinline__ const float* E(const ColDev& C) { return C.Ebff; }
  static __device__ __forceinline__ float wm2(const ColDev& C, int m) { return C.wm2f[m]; }
  static __device__ __forceinline__ float i2mu(const ColDev& C, int m) { return C.inv2muf[m]; }
};

// chi and S for one 64-frequency chunk and KG consecutive depths:
// one wave, one lane per frequency, the depths unrolled in registers; the
// windows overlapping the chunk are visited one after the other, so each
// transition's coefficients for all the wave's depths come in one scalar load.
// Explicit FMAs keep the arithmetic identical for every depth-group size.
// The sums are FP64 in both forms (the FP32 form reads FP32 copies of the
// n-independent tables) and only chi and S leave rounded to R: near
// population inversion a line can cancel most of the background
// opacity, and the FP32 form's preconditioner is nearly singular in
// scattering-dominated lines, so rounding before the cancellation shows up as
// noise in the finite-difference product (on MI355X an FP64 FMA issues at the
// rate of a non-packed FP32 one, so this costs no extra issue slots).
// KG (depths per wave) is a launch shape the plan tuner chooses among 4, 8, 16.
// FLY (FP32 form only): B_nu(T) and e^{-h nu/kT} made here rather than read
// from the tables (columns without a caller emissivity).  A compile-time
// choice, taken once per wave by the callers: as a branch per depth, the
// table loads of the other side made the compiler wait for every load and
// store in flight before each exponential.
//
// CACHED: the depth-independent inputs of every depth group (gamma = 2 h
// nu^3 / c^2 and h nu / k of the lane's frequency, and the cross-sections
// of the chunk's edges, all of them) come from a per-wave copy in LDS made
// once before the sweep (opacity_cache_fill) instead of a vector load per
// group and edge, each of which made the wave wait for every load and store
// it had in flight.  The same values, so the same bits.
constexpr int kEdgeCache = 6;  // edges a chunk may have to use the LDS copy
template <typename R>
struct OpacityCache {
  static constexpr int kBytes = kWave * 8 + kWave * 4 + kEdgeCache * kWave * (int)sizeof(R);
  static __device__ __forceinline__ double* gam(char* b) { return reinterpret_cast<double*>(b); }
  static __device__ __forceinline__ float* hnuk(char* b) {
    return reinterpret_cast<float*>(b + kWave * 8);
  }
  static __device__ __forceinline__ R* al(char* b) {
    return reinterpret_cast<R*>(b + kWave * 12);
  }
};

template <typename R, int KG, bool FLY, bool CACHED>
__device__ __forceinline__ void opacity_group(const ColDev& C, int chunk, int k0, int nz, int nnu,
                                              bool fin, int fc, const R* __restrict__ Vt,
                                              const double* __restrict__ coef, int ntr,
                                              R (&cx)[KG], R (&sx)[KG], char* cache, int lane);

// Whether a column's opacity in precision R is made with FLY (see above).
template <typename R>
__device__ __forceinline__ bool opacity_fly(const ColDev& C) {
  return sizeof(R) == sizeof(float) && !C.bg_eta;
}

// nsplit waves share a tile's depth groups (round-robin), so that a launch
// over few tiles (one large column) still fills the chip; every depth group is
// computed the same way whichever wave takes it.
template <typename R, int KG>
__global__ __launch_bounds__(256) void k_opacity(const ColDev* __restrict__ cols,
                                                 const Tile* __restrict__ tiles, int ntiles,
                                                 int nsplit) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // a column's chunks and depth groups on one XCD (shared coefficients)
  const int wid = xcd_item(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
  const int tid = wid / nsplit, part = wid - tid * nsplit;
  if (tid >= ntiles) return;
  const int col = uni(tiles[tid].col);
  const int chunk = uni(tiles[tid].chunk);
  const ColDev& C = cols[col];
  if (uni(C.st->mode) == kModeIdle) return;
  if (uni(C.st->cur_prec) != (sizeof(R) == sizeof(float) ? NLTE_FP32_FORM : NLTE_FP64)) return;
  const int nz = uni(C.nz), nnu = uni(C.nnu);
  const int f = chunk * kWave + lane;
  const bool fin = f < nnu;
  const int fc = fin ? f : nnu - 1;
  const R* __restrict__ Vt = FTab<R>::V(C);
  const double* __restrict__ coef = (const double*)C.coef;
  const int ntr = uni(C.ntr);
  auto groups = [&](auto fly) {
    for (int k0 = part * KG; k0 < nz; k0 += nsplit * KG) {
      R cx[KG], sx[KG];
      opacity_group<R, KG, decltype(fly)::value, false>(C, chunk, k0, nz, nnu, fin, fc, Vt, coef,
                                                        ntr, cx, sx, nullptr, 0);
    }
  };
  if (opacity_fly<R>(C))
    groups(std::integral_constant<bool, sizeof(R) == sizeof(float)>{});
  else
    groups(std::false_type{});
}

template <typename R, int KG, bool FLY, bool CACHED>
__device__ __forceinline__ void opacity_group(const ColDev& C, int chunk, int k0, int nz, int nnu,
                                              bool fin, int fc, const R* __restrict__ Vt,
                                              const double* __restrict__ coef, int ntr,
                                              R (&cx)[KG], R (&sx)[KG], char* cache, int lane) {
  static_assert(!FLY || sizeof(R) == sizeof(float), "B and E on the fly: FP32 form only");
  static_assert(!CACHED || FLY, "the LDS copy serves the on-the-fly form");
  double chi[KG], et[KG];
#pragma unroll
  for (int i = 0; i < KG; ++i) {
    chi[i] = 0.0;
    et[i] = 0.0;
  }
  // lines: chi += V c0, et += V c1.  The chunk's transition lists and the
  // transitions' windows are set up before any evaluation and read through
  // the scalar cache (ldc): generic loads of them became vector loads whose
  // waits drained every load and store the wave had in flight.
  const int l0 = ldc(C.ch_lptr + chunk), l1 = ldc(C.ch_lptr + chunk + 1);
  for (int j = l0; j < l1; ++j) {
    const int t = ldc(C.ch_line + j);
    const TrDev* T = C.tr + t;
    const int wlo = ldc(&T->wlo), wl = ldc(&T->whi) - wlo;
    const int q = fc - wlo;
    const bool in = q >= 0 && q < wl;
    const R* vrow = Vt + ldc(&T->voff) + (in ? q : 0);
    const double* ct = coef + ((size_t)t * nz + k0) * 2;
    R v[KG];
#pragma unroll
    for (int i = 0; i < KG; ++i) {
      const int k = min(k0 + i, nz - 1);
      v[i] = ldg(vrow + (size_t)k * wl);
    }
#pragma unroll
    for (int i = 0; i < KG; ++i) {
      const int k = min(k0 + i, nz - 1) - k0;
      const double vi = in ? (double)v[i] : 0.0;
      chi[i] = fmar(vi, ldc(ct + 2 * k), chi[i]);
      et[i] = fmar(vi, ldc(ct + 2 * k + 1), et[i]);
    }
  }
  // edges: A1 = sum alpha c0, A2 = sum alpha c1
  double A1[KG], A2[KG];
#pragma unroll
  for (int i = 0; i < KG; ++i) {
    A1[i] = 0.0;
    A2[i] = 0.0;
  }
  const int e0 = ldc(C.ch_eptr + chunk), e1 = ldc(C.ch_eptr + chunk + 1);
  for (int j = e0; j < e1; ++j) {
    const int t = ldc(C.ch_edge + j);
    double al;
    if (CACHED) {
      al = (double)OpacityCache<R>::al(cache)[(j - e0) * kWave + lane];
    } else {
      const TrDev* T = C.tr + t;
      const int wlo = ldc(&T->wlo), whi = ldc(&T->whi);
      al = (fc >= wlo && fc < whi) ? (double)ldg(Vt + ldc(&T->voff) + (fc - wlo)) : 0.0;
    }
    const double* ct = coef + ((size_t)t * nz + k0) * 2;
#pragma unroll
    for (int i = 0; i < KG; ++i) {
      const int k = min(k0 + i, nz - 1) - k0;
      A1[i] = fmar(al, ldc(ct + 2 * k), A1[i]);
      A2[i] = fmar(al, ldc(ct + 2 * k + 1), A2[i]);
    }
  }
  // background, source function
  const double gam = CACHED ? OpacityCache<R>::gam(cache)[lane] : ldg(C.gam + fc);
  const double* cb = coef + ((size_t)ntr * nz + k0) * 2;
  const double* cs = coef + ((size_t)(ntr + 1) * nz + k0) * 2;
  const bool sca = C.has_sca, bf = C.nbf > 0;
  R* __restrict__ xs = reinterpret_cast<R*>(C.XS);
  // the FP32 tables share the scratch's padded row pitch; the FP64 ones
  // (and the lagged J) keep rows of nnu
  const int fp = uni(C.fp), tp = sizeof(R) == sizeof(float) ? fp : nnu;
  // FP32 form: B_nu(T) and exp(-h nu / kT) made here in FP32 (n-independent,
  // like the FP32 tables they replace) unless the caller gave the emissivity
  constexpr bool fly = FLY;
  const float hnuk = CACHED ? OpacityCache<R>::hnuk(cache)[lane]
                            : fly ? (float)(kH / kK * ldg(C.nu + fc)) : 0.0f;
  const float gamf = (float)gam;
#pragma unroll
  for (int i = 0; i < KG; ++i) {
    const int k = min(k0 + i, nz - 1);
    const size_t kf = (size_t)k * nnu + fc, kt = (size_t)k * tp + fc, kx = (size_t)k * fp + fc;
    double B, E;
    if (fly) {
      const float Ef = __expf(-hnuk * __builtin_amdgcn_rcpf((float)ldc(C.T + k)));
      E = (double)Ef;
      B = (double)(gamf * Ef * __builtin_amdgcn_rcpf(1.0f - Ef));
    } else {
      B = (double)ldg(FTab<R>::B(C) + kt);
      E = bf ? (double)ldg(FTab<R>::E(C) + kt) : 0.0;
    }
    if (!bf) E = 0.0;
    const double EA2 = E * A2[i];
    const double X = (ldc(cb + 2 * (k - k0)) + chi[i]) + (A1[i] - EA2);
    double eta = fmar(ldc(cb + 2 * (k - k0) + 1), B, gam * (et[i] + EA2));
    if (sca) eta = fmar(ldc(cs + 2 * (k - k0)), ldg(C.Jdag + kf), eta);
    cx[i] = (R)X;
    sx[i] = (R)(eta / X);
    if (fin && k0 + i < nz) {
      stg(xs + 2 * kx, cx[i]);
      stg(xs + 2 * kx + 1, sx[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// formal solution kernel
// ---------------------------------------------------------------------------
// R: arithmetic of the depth recursion (double, or float for the FP32 form;
// J and the derivatives leave in double).  PM: Newton mode (also the local
// intensity derivatives of App. A.2).  NMU: angles per hemisphere.
// One wave per 64-frequency chunk, one lane per frequency, all 2 NMU rays in
// registers.  The first sweep (ingoing rays, top -> bottom) parks its share
// of J in a scratch row; the second (outgoing rays, bottom -> top) writes J.
// The depth-contiguous outputs leave through the per-wave LDS staging tiles
// of nlte_kernels.h.

// Depth-group size of the opacity made inside the first sweep.
constexpr int kFusedDepths = 4;
// FP32 tile groups at least this large (enough chunk waves to fill the chip)
// make their opacity inside the formal-solution kernel; smaller ones, and the
// FP64 recursion (whose registers leave less room), keep the depth-parallel
// opacity kernel.  The opacity arithmetic does not depend on the depth-group
// size, so both give the same bits.
constexpr int kFuseMinTiles = 4096;
// Depths per LDS staging tile: a flush writes, for each frequency of the
// chunk, that many consecutive FP64 depths.
template <typename R, bool PM> struct StageDepths {
  static constexpr int value = PM ? 4 : 8;
};
// Depths per operand block of the sweeps: 4 in FP32 (more loads in flight
// per wait), 2 in FP64, whose larger registers cost occupancy instead
// (batch6 FP64 F-only 10.15 -> 10.00 ms, solve 1167 -> 1133 ms with 2; the
// FP32 form is slower with 2: 5.63 -> 5.81 ms).
template <typename R> struct DepthBlock {
  static constexpr int value = sizeof(R) == sizeof(float) ? 4 : 2;
};

// The LDS copy of OpacityCache for one wave: each lane writes, and later
// reads, only its own entries, so no barrier is needed.  False (nothing
// written) if the chunk has more edges than the copy holds.
template <typename R>
__device__ __forceinline__ bool opacity_cache_fill(const ColDev& C, int chunk, int fc, int lane,
                                                   const R* __restrict__ Vt, char* cache) {
  const int e0 = ldc(C.ch_eptr + chunk), e1 = ldc(C.ch_eptr + chunk + 1);
  if (e1 - e0 > kEdgeCache) return false;
  OpacityCache<R>::gam(cache)[lane] = ldg(C.gam + fc);
  OpacityCache<R>::hnuk(cache)[lane] = (float)(kH / kK * ldg(C.nu + fc));
  for (int j = e0; j < e1; ++j) {
    const TrDev* T = C.tr + ldc(C.ch_edge + j);
    const int wlo = ldc(&T->wlo), whi = ldc(&T->whi);
    OpacityCache<R>::al(cache)[(j - e0) * kWave + lane] =
        (fc >= wlo && fc < whi) ? ldg(Vt + ldc(&T->voff) + (fc - wlo)) : (R)0;
  }
  return true;
}

// cache: this wave's LDS for OpacityCache (F-mode launches that make their
// opacity here), or NULL.
template <typename R, bool PM, int NMU>
__device__ __forceinline__ void formal_tile(const ColDev& C, int chunk, int lane, double* tile,
                                            bool fused, char* cache) {
  constexpr int KF = StageDepths<R, PM>::value;
  double* tJ = tile;
  double* tX = tile + KF * kWave;
  double* tE = tile + 2 * KF * kWave;
  const int f0 = chunk * kWave;
  const int nz = C.nz, nnu = C.nnu, fp = C.fp, zp = C.zp;
  const int f = chunk * kWave + lane;
  const bool fin = f < nnu;
  const int fc = fin ? f : nnu - 1;
  const double* __restrict__ dzt = (const double*)C.coef + ((size_t)(C.ntr + 1) * nz) * 2 + 1;  // stride 2
  // [nz][nnu][2]: chi, S (in the fused variant written by the first sweep)
  const R* xs = reinterpret_cast<const R*>(C.XS);
  // [nz][nnu] ingoing half of J, stored in the recursion's precision (the
  // angle sums themselves are FP64)
  R* __restrict__ jm = reinterpret_cast<R*>(C.Jm);
  R* __restrict__ dxs = reinterpret_cast<R*>(C.Dchi);           // [nz][nnu]
  R* __restrict__ des = reinterpret_cast<R*>(C.Deta);           // [nz][nnu]

  R wm2[NMU], i2mu[NMU], mu2[NMU];
  double wm2d[NMU];
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    wm2[m] = FTab<R>::wm2(C, m);
    i2mu[m] = FTab<R>::i2mu(C, m);
    mu2[m] = (R)(1.0 / C.inv2mu[m]);
    wm2d[m] = C.wm2[m];
  }

  // Both sweeps take their per-depth operands DepthBlock depths at a time,
  // loaded one block ahead (depth indices clamped into the column, so every
  // load is unconditional): a wave has that many steps of arithmetic in hand
  // while a block's loads are in flight.
  constexpr int U = DepthBlock<R>::value;

  // ---- sweep 1: ingoing rays, top -> bottom (I- = 0 at the top) ----
  R I[NMU];
#pragma unroll
  for (int m = 0; m < NMU; ++m) I[m] = (R)0;
  R chi_p = (R)0, S_p = (R)0;
  if (fin) {
    stg(jm + f, (R)0);
    if (PM) {
      stg(dxs + f, (R)0);
      stg(des + f, (R)0);
    }
  }
  auto down_step = [&](int k, R chi, R S, R dz) {
    const R base = dz * (chi_p + chi);
    const R rb = PL<R>::div((R)1, base);
    const R dS = S - S_p;
    double jac = 0.0;
    R sa = (R)0, sc = (R)0;
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      const R Iup = I[m];
      const R x = base * i2mu[m];
      R e, q, a, bx;
      seg_coef<R, PM>(x, rb, mu2[m], e, q, a, bx);
      I[m] = fmar(e, Iup, fmar(q, S_p, a * dS));
      jac = fmar(wm2d[m], (double)I[m], jac);
      if (PM) {
        // c_chi, c_eta of App. A.2 (ingoing ray, segment k-1 -> k)
        sa += wm2[m] * a;
        sc += (wm2[m] * i2mu[m]) * (e * (S_p - Iup) - (S_p - S) * bx);
      }
    }
    if (fin) {
      const size_t kf = (size_t)k * fp + f;
      stg(jm + kf, (R)jac);
      if (PM) {
        const R rc = PL<R>::div((R)1, chi);
        stg(dxs + kf, -(S * rc) * sa + dz * sc);
        stg(des + kf, sa * rc);
      }
    }
    chi_p = chi;
    S_p = S;
  };
  if (fused) {
    // chi and S of kFusedDepths depths at a time from the opacity, made here
    // (and kept for the second sweep): the table reads of one wave overlap
    // the recursion arithmetic of the others
    const R* __restrict__ Vt = FTab<R>::V(C);
    const double* __restrict__ coef = (const double*)C.coef;
    const int ntr = C.ntr;
    auto sweep = [&](auto fly, auto cached) {
      for (int k0 = 0; k0 < nz; k0 += kFusedDepths) {
        R gc[kFusedDepths], gs[kFusedDepths], gd[kFusedDepths];
#pragma unroll
        for (int u = 0; u < kFusedDepths; ++u)
          gd[u] = (R)ldc(dzt + 2 * max(min(k0 + u, nz - 1) - 1, 0));
        opacity_group<R, kFusedDepths, decltype(fly)::value, decltype(cached)::value>(
            C, chunk, k0, nz, nnu, fin, fc, Vt, coef, ntr, gc, gs, cache, lane);
#pragma unroll
        for (int u = 0; u < kFusedDepths; ++u) {
          const int k = k0 + u;
          if (k == 0) {
            chi_p = gc[0];
            S_p = gs[0];
          } else if (k < nz) {
            down_step(k, gc[u], gs[u], gd[u]);
          }
        }
      }
    };
    using FlyOk = std::integral_constant<bool, sizeof(R) == sizeof(float)>;
    if (opacity_fly<R>(C)) {
      if (FlyOk::value && cache && opacity_cache_fill<R>(C, chunk, fc, lane, Vt, cache))
        sweep(FlyOk{}, FlyOk{});
      else
        sweep(FlyOk{}, std::false_type{});
    } else {
      sweep(std::false_type{}, std::false_type{});
    }
  } else {
    chi_p = ldg(xs + 2 * (size_t)fc);
    S_p = ldg(xs + 2 * (size_t)fc + 1);
    // segment k-1 -> k has thickness dz[k-1]
    R cc[U], cs[U], nc[U], ns[U], cd[U], nd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = min(1 + u, nz - 1);
      const size_t kf = (size_t)k * fp + fc;
      cc[u] = ldg(xs + 2 * kf);
      cs[u] = ldg(xs + 2 * kf + 1);
      cd[u] = (R)ldc(dzt + 2 * max(k - 1, 0));
    }
    for (int k0 = 1; k0 < nz; k0 += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = min(k0 + U + u, nz - 1);
        const size_t kf = (size_t)k * fp + fc;
        nc[u] = ldg(xs + 2 * kf);
        ns[u] = ldg(xs + 2 * kf + 1);
        nd[u] = (R)ldc(dzt + 2 * max(k - 1, 0));
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 + u < nz) down_step(k0 + u, cc[u], cs[u], cd[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cc[u] = nc[u];
        cs[u] = ns[u];
        cd[u] = nd[u];
      }
    }
  }

  // ---- sweep 2: outgoing rays, bottom -> top (I+ = B at the bottom) ----
  R chi_n = chi_p, S_n = S_p;
  {
    const size_t kf = (size_t)(nz - 1) * fp + fc;
    const double Bd = ldg(C.Bnu + (size_t)(nz - 1) * nnu + fc);
    const R Bb = (R)Bd;
    double jp = 0.0;
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      I[m] = Bb;
      jp = fmar(wm2d[m], (double)Bb, jp);
    }
    stage_put<KF>(tJ, nz - 1, lane, (double)ldg(jm + kf) + jp);
    if (PM) {  // bottom: ingoing-ray derivatives only
      stage_put<KF>(tX, nz - 1, lane, (double)ldg(dxs + kf));
      stage_put<KF>(tE, nz - 1, lane, (double)ldg(des + kf));
    }
    if ((nz - 1) % KF == 0) {
      stage_flush<KF>(tJ, C.JT, nz - 1, nz, zp, f0, nnu, lane);
      if (PM) {
        stage_flush<KF>(tX, C.DchiT, nz - 1, nz, zp, f0, nnu, lane);
        stage_flush<KF>(tE, C.DetaT, nz - 1, nz, zp, f0, nnu, lane);
      }
    }
  }
  auto up_step = [&](int k, R chi, R S, double jm_k, R dX_k, R dE_k, R dz) {
    const R base = dz * (chi + chi_n);
    const R rb = PL<R>::div((R)1, base);
    const R dS = S - S_n;
    double jp = 0.0;
    R sa = (R)0, sc = (R)0;
#pragma unroll
    for (int m = 0; m < NMU; ++m) {
      const R Iup = I[m];
      const R x = base * i2mu[m];
      R e, q, a, bx;
      seg_coef<R, PM>(x, rb, mu2[m], e, q, a, bx);
      I[m] = fmar(e, Iup, fmar(q, S_n, a * dS));
      jp = fmar(wm2d[m], (double)I[m], jp);
      if (PM) {
        // a_chi, a_eta of App. A.2 (outgoing ray, segment k+1 -> k)
        sa += wm2[m] * a;
        sc += (wm2[m] * i2mu[m]) * (e * (S_n - Iup) - (S_n - S) * bx);
      }
    }
    stage_put<KF>(tJ, k, lane, jm_k + jp);
    if (PM) {
      const R rc = PL<R>::div((R)1, chi);
      stage_put<KF>(tX, k, lane, (double)dX_k + (double)(-(S * rc) * sa + dz * sc));
      stage_put<KF>(tE, k, lane, (double)dE_k + (double)(sa * rc));
    }
    if (k % KF == 0) {
      stage_flush<KF>(tJ, C.JT, k, nz, zp, f0, nnu, lane);
      if (PM) {
        stage_flush<KF>(tX, C.DchiT, k, nz, zp, f0, nnu, lane);
        stage_flush<KF>(tE, C.DetaT, k, nz, zp, f0, nnu, lane);
      }
    }
    chi_n = chi;
    S_n = S;
  };
  {
    // block b covers depths k0, k0 - 1, ..., k0 - U + 1 (clamped at 0)
    // segment k -> k+1 has thickness dz[k]
    R cc[U], cs[U], nc[U], ns[U], cx[U], ce[U], nx[U], ne[U], cd[U], nd[U];
    double cj[U], nj[U];
    auto load = [&](int k0, R* c_, R* s_, double* j_, R* x_, R* e_, R* d_) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = max(k0 - u, 0);
        const size_t kf = (size_t)k * fp + fc;
        d_[u] = (R)ldc(dzt + 2 * k);
        c_[u] = ldg(xs + 2 * kf);
        s_[u] = ldg(xs + 2 * kf + 1);
        j_[u] = (double)ldg(jm + kf);
        if (PM) {
          x_[u] = ldg(dxs + kf);
          e_[u] = ldg(des + kf);
        } else {
          x_[u] = (R)0;
          e_[u] = (R)0;
        }
      }
    };
    load(nz - 2, cc, cs, cj, cx, ce, cd);
    for (int k0 = nz - 2; k0 >= 0; k0 -= U) {
      load(k0 - U, nc, ns, nj, nx, ne, nd);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 - u >= 0) up_step(k0 - u, cc[u], cs[u], cj[u], cx[u], ce[u], cd[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cd[u] = nd[u];
        cc[u] = nc[u];
        cs[u] = ns[u];
        cj[u] = nj[u];
        cx[u] = nx[u];
        ce[u] = ne[u];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// depth-parallel formal solution (columns created with NLTE_DEPTH_SCAN)
// ---------------------------------------------------------------------------
// One workgroup per frequency, one thread per depth.  Along a ray the
// piecewise-linear scheme is an affine recursion over depth,
//   downwards  I_k = e I_{k-1} + (a S_k + b S_{k-1}),
//   upwards    I_k = e I_{k+1} + (a S_k + b S_{k+1}),
// with the same e, a, b for a segment in both directions (they depend on
// its optical thickness only), so each segment's coefficients are computed
// once.  Composing affine maps is associative: each direction is a parallel
// prefix over depth (shuffles within a wave, one combination across the
// workgroup's waves).  All maps have e >= 0 and, for S >= 0, s >= 0, so the
// scan adds no cancellation.

// a, b, e = 1 - a - b and b/x of a segment (Appendix A.1).
template <typename R>
__device__ __forceinline__ void pl_coefs(R x, R& a, R& b, R& e, R& bx) {
  if (x < PL<R>::kSwitch) {
    R pa, pb;
    horner_ab<R, 1, PL<R>::kTermsAB>(x, pa, pb);
    a = pa * x;
    b = pb * x;
    e = (R)1 - a - b;
    bx = pb;
  } else {
    e = PL<R>::ex(x);
    const R t1 = PL<R>::div((R)1 - e, x);
    a = (R)1 - t1;
    b = t1 - e;
    bx = PL<R>::div(b, x);
  }
}

// Inclusive scans of affine maps (e, s): I -> e I + s.  Downward: thread t
// ends with M_t o ... o M_0; upward: with M_t o ... o M_last.
template <typename R>
__device__ __forceinline__ void scan_down(R& e, R& s, R* le, R* ls) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const R pe = __shfl_up(e, d), ps = __shfl_up(s, d);
    if (lane >= d) {
      s = fmar(e, ps, s);
      e = e * pe;
    }
  }
  if (lane == kWave - 1) {
    le[wave] = e;
    ls[wave] = s;
  }
  __syncthreads();
  R ce = (R)1, cs = (R)0;
  for (int w = 0; w < wave; ++w) {
    cs = fmar(le[w], cs, ls[w]);
    ce = le[w] * ce;
  }
  s = fmar(e, cs, s);
  e = e * ce;
  __syncthreads();
}

template <typename R>
__device__ __forceinline__ void scan_up(R& e, R& s, R* le, R* ls) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const R pe = __shfl_down(e, d), ps = __shfl_down(s, d);
    if (lane + d < kWave) {
      s = fmar(e, ps, s);
      e = e * pe;
    }
  }
  if (lane == 0) {
    le[wave] = e;
    ls[wave] = s;
  }
  __syncthreads();
  R ce = (R)1, cs = (R)0;
  for (int w = nw - 1; w > wave; --w) {
    cs = fmar(le[w], cs, ls[w]);
    ce = le[w] * ce;
  }
  s = fmar(e, cs, s);
  e = e * ce;
  __syncthreads();
}

// 64 workgroups per chunk tile (one per frequency of the chunk).
template <typename R, bool PM, int NMU>
__global__ __launch_bounds__(kScanThreads) void k_formal_scan(const ColDev* __restrict__ cols,
                                                              const Tile* __restrict__ tiles,
                                                              int ntiles) {
  const int b = xcd_item(blockIdx.x, gridDim.x);  // a column's frequencies on one XCD
  const int tile = b >> 6, fl = b & 63;
  if (tile >= ntiles) return;
  const int col = uni(tiles[tile].col), chunk = uni(tiles[tile].chunk);
  const ColDev& C = cols[col];
  const int mode = uni(C.st->mode);
  if (mode != (PM ? kModeNewton : kModeF)) return;
  if (uni(C.st->cur_prec) != (sizeof(R) == sizeof(float) ? NLTE_FP32_FORM : NLTE_FP64)) return;
  const int nz = uni(C.nz), nnu = uni(C.nnu);
  const int f = chunk * kWave + fl;
  if (f >= nnu) return;
  const int t = threadIdx.x;
  const bool in = t < nz;
  const int k = in ? t : nz - 1;

  __shared__ R sx[kScanThreads], ss[kScanThreads];
  __shared__ R se[kScanThreads], sa[kScanThreads], sb[kScanThreads], sbx[kScanThreads];
  __shared__ R sin_[kScanThreads], sout[kScanThreads];
  __shared__ R le[kScanThreads / kWave], ls[kScanThreads / kWave];

  const R* __restrict__ xs = reinterpret_cast<const R*>(C.XS);
  const double* __restrict__ dzt = C.coef + ((size_t)(C.ntr + 1) * nz) * 2 + 1;  // stride 2
  const size_t kf = (size_t)k * uni(C.fp) + f;
  const R chi = ldg(xs + 2 * kf), S = ldg(xs + 2 * kf + 1);
  sx[t] = chi;
  ss[t] = S;
  __syncthreads();
  const bool up_seg = in && t > 0;       // segment (t-1, t) exists
  const bool dn_seg = in && t + 1 < nz;  // segment (t, t+1) exists
  const R chi_p = up_seg ? sx[t - 1] : chi, S_p = up_seg ? ss[t - 1] : S;
  const R S_n = dn_seg ? ss[t + 1] : S;
  const R dz_p = up_seg ? (R)ldg(dzt + 2 * (t - 1)) : (R)0;
  const R dz_n = dn_seg ? (R)ldg(dzt + 2 * t) : (R)0;
  const R base = dz_p * (chi_p + chi);  // optical thickness of (t-1, t) times 2 mu
  const R Bb = (R)ldg(C.Bnu + (size_t)(nz - 1) * nnu + f);
  const R rc = PM ? PL<R>::div((R)1, chi) : (R)0;

  double jac = 0.0, dX = 0.0, dE = 0.0;
#pragma unroll
  for (int m = 0; m < NMU; ++m) {
    const R i2m = FTab<R>::i2mu(C, m);
    R a, b, e, bx;
    pl_coefs<R>(base * i2m, a, b, e, bx);
    se[t] = e;
    sa[t] = a;
    sb[t] = b;
    if (PM) sbx[t] = bx;
    __syncthreads();
    // segment (t, t+1) as computed by thread t + 1
    const R e2 = dn_seg ? se[t + 1] : (R)0, a2 = dn_seg ? sa[t + 1] : (R)0;
    const R b2 = dn_seg ? sb[t + 1] : (R)0, bx2 = (PM && dn_seg) ? sbx[t + 1] : (R)0;
    // downward map at t: I_0 = 0 at the top
    R fe = (R)1, fs = (R)0;
    if (in) {
      fe = up_seg ? e : (R)0;
      fs = up_seg ? fmar(a, S, b * S_p) : (R)0;
    }
    // upward map at t: I = B at the bottom
    R ge = (R)1, gs = (R)0;
    if (in) {
      ge = dn_seg ? e2 : (R)0;
      gs = dn_seg ? fmar(a2, S, b2 * S_n) : Bb;
    }
    scan_down<R>(fe, fs, le, ls);
    scan_up<R>(ge, gs, le, ls);
    const double w = FTab<double>::wm2(C, m);
    jac = fmar(w, (double)fs + (double)gs, jac);
    if (PM) {
      sin_[t] = fs;
      sout[t] = gs;
      __syncthreads();
      const R i2 = i2m;
      if (up_seg) {  // c_chi, c_eta of App. A.2 (ingoing ray, segment t-1 -> t)
        const R Iup = sin_[t - 1];
        const R cchi = -(S * rc) * a + dz_p * i2 * (e * (S_p - Iup) - (S_p - S) * bx);
        dX = fmar(w, (double)cchi, dX);
        dE = fmar(w, (double)(a * rc), dE);
      }
      if (dn_seg) {  // a_chi, a_eta (outgoing ray, segment t+1 -> t)
        const R Iup = sout[t + 1];
        const R achi = -(S * rc) * a2 + dz_n * i2 * (e2 * (S_n - Iup) - (S_n - S) * bx2);
        dX = fmar(w, (double)achi, dX);
        dE = fmar(w, (double)(a2 * rc), dE);
      }
    }
    __syncthreads();  // the coefficient and intensity rows are rewritten for the next angle
  }
  if (in) {
    const size_t fk = (size_t)f * uni(C.zp) + t;
    stg(C.JT + fk, jac);
    if (PM) {
      stg(C.DchiT + fk, dX);
      stg(C.DetaT + fk, dE);
    }
  }
}

template <typename R, bool PM>
static void launch_formal_scan_mu(int nmu, hipStream_t s, const ColDev* cols, const Tile* tiles,
                                  int ntiles) {
  const int blocks = ntiles * kWave;
  switch (nmu) {
#define NLTE_SCAN_CASE(M) \
  case M: k_formal_scan<R, PM, M><<<blocks, kScanThreads, 0, s>>>(cols, tiles, ntiles); break;
    NLTE_SCAN_CASE(1) NLTE_SCAN_CASE(2) NLTE_SCAN_CASE(3) NLTE_SCAN_CASE(4)
    NLTE_SCAN_CASE(5) NLTE_SCAN_CASE(6) NLTE_SCAN_CASE(7) NLTE_SCAN_CASE(8)
#undef NLTE_SCAN_CASE
    default: break;
  }
}

// One launch per (precision, angle count, mode) present in a step, over that
// group's tiles; a wave whose column is idle or in the other mode returns.
template <typename R, bool PM, int NMU>
__global__ __launch_bounds__(256) void k_formal(const ColDev* __restrict__ cols,
                                                const Tile* __restrict__ tiles, int ntiles,
                                                int fused, const Tile* __restrict__ mlist,
                                                const int* __restrict__ mcount) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // the chunks of a column are consecutive tiles: keeping them on one XCD
  // lets them share the column's level coefficients and the table lines
  // their rows have in common in that XCD's L2
  Tile t;
  if (!pick_tile(tiles, ntiles, mlist, mcount, wave, t)) return;
  const int col = t.col, chunk = t.chunk;
  const ColDev& C = cols[col];
  const int mode = uni(C.st->mode);
  if (mode != (PM ? kModeNewton : kModeF)) return;
  if (uni(C.st->cur_prec) != (sizeof(R) == sizeof(float) ? NLTE_FP32_FORM : NLTE_FP64)) return;
  constexpr int KF = StageDepths<R, PM>::value;
  constexpr int NT = PM ? 3 : 1;  // staged outputs: J (and the two derivatives)
  // per wave: the staging tiles, then (F-mode launches that make their
  // opacity) the OpacityCache copy
  constexpr bool kCache = !PM && sizeof(R) == sizeof(float);
  const int per_wave = NT * KF * kWave * 8 + (kCache && fused ? OpacityCache<R>::kBytes : 0);
  extern __shared__ double stage[];
  char* mine = reinterpret_cast<char*>(stage) + wave * per_wave;
  formal_tile<R, PM, NMU>(C, chunk, lane, reinterpret_cast<double*>(mine), fused != 0,
                          kCache && fused ? mine + NT * KF * kWave * 8 : nullptr);
}

template <typename R, bool PM>
static void launch_formal_mu(int nmu, int wpb, hipStream_t s, const ColDev* cols,
                             const Tile* tiles, int ntiles, int fused,
                             const Tile* mlist = nullptr, const int* mcount = nullptr) {
  const int blocks = (ntiles + wpb - 1) / wpb;
  constexpr bool kCache = !PM && sizeof(R) == sizeof(float);
  const size_t lds = (size_t)wpb * ((PM ? 3 : 1) * StageDepths<R, PM>::value * kWave * sizeof(double) +
                                    (kCache && fused ? OpacityCache<R>::kBytes : 0));
  switch (nmu) {
#define NLTE_FORMAL_CASE(M) \
  case M: \
    k_formal<R, PM, M><<<blocks, 64 * wpb, lds, s>>>(cols, tiles, ntiles, fused, mlist, mcount); \
    break;
    NLTE_FORMAL_CASE(1) NLTE_FORMAL_CASE(2) NLTE_FORMAL_CASE(3) NLTE_FORMAL_CASE(4)
    NLTE_FORMAL_CASE(5) NLTE_FORMAL_CASE(6) NLTE_FORMAL_CASE(7) NLTE_FORMAL_CASE(8)
#undef NLTE_FORMAL_CASE
    default: break;
  }
}

// ---------------------------------------------------------------------------
// rate integrals (Eqs. Rij, Rji): one lane per depth, sequential sums over
// the frequencies of a piece for every transition covering it (depth-
// contiguous operands, so every load of a wave is one contiguous run).
// Lines: sum cw V J.  Edges: sum cw alpha J and sum cw alpha exp(-h nu/kT) J
// (the J part of R_ul without its depth factor).  A block loads J (and
// e^{-h nu/kT}) once per frequency for all its transitions.  Every term is
// positive and a piece holds at most kSegLen frequencies, so each partial
// sum stays within kSegLen roundings (below 6e-14 relative); the assembly
// adds the pieces of a transition in frequency order.
// ---------------------------------------------------------------------------
// TB: line-table precision (float for FP32-form evaluations).  J stays FP64
// here: in the FP32 form a J rounded to FP32 before these sums sets a noise
// floor on F that doubled the share of columns needing the FP64 fallback.
template <typename TB, int NL, int NE, bool SC>
__device__ __forceinline__ void rates_block(const ColDev& C, const RItem& it, int k,
                                            const TB* __restrict__ VTt, const TB* __restrict__ EbfTt) {
  // wave-uniform per-frequency data: scalar loads (SC) or vector loads
  auto rd = [](const double* p) { return SC ? ldc(p) : ldg(p); };
  const int nz = C.nz, zp = C.zp, f0 = it.f0, nf = it.f1 - it.f0;
  const TB* vl[NL > 0 ? NL : 1];      // line V at f0, this lane's depth (rows of nz)
  const double* cl[NL > 0 ? NL : 1];  // line rate weights at f0
  const double* ae[NE > 0 ? NE : 1];  // edge cross-sections at f0
  const double* ce[NE > 0 ? NE : 1];  // edge rate weights at f0
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const TrDev& T = C.tr[it.t[i]];
    const int wo = f0 - uni(T.wlo);
    vl[i] = VTt + uni(T.voff) + (size_t)wo * nz + k;
    cl[i] = C.cw + uni(T.cwoff) + wo;
  }
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const TrDev& T = C.tr[it.t[NL + i]];
    const int wo = f0 - uni(T.wlo);
    ae[i] = C.V + uni(T.voff) + wo;
    ce[i] = C.cw + uni(T.cwoff) + wo;
  }
  const double* __restrict__ J = C.JT + (size_t)f0 * zp + k;
  const TB* __restrict__ E = NE > 0 ? EbfTt + (size_t)f0 * zp + k : nullptr;
  double sl[NL > 0 ? NL : 1], s1[NE > 0 ? NE : 1], s2[NE > 0 ? NE : 1];
#pragma unroll
  for (int i = 0; i < NL; ++i) sl[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NE; ++i) s1[i] = s2[i] = 0.0;
  // the rate weights and the edges' cross-sections depend on the frequency
  // only.  With SC they are scalar loads (ldc), which leave the vector loads
  // of J and V in flight (generic loads wait for every load issued before
  // them): faster where many waves share a CU; a launch of a few hundred
  // waves (one deep column) is faster with vector loads, which it keeps.
#pragma unroll 4
  for (int q = 0; q < nf; ++q) {
    const size_t o = (size_t)q * zp;
    const double j = ldg(J + o);
#pragma unroll
    for (int i = 0; i < NL; ++i) sl[i] = fma(rd(cl[i] + q) * (double)ldg(vl[i] + (size_t)q * nz), j, sl[i]);
    if (NE > 0) {
      const double e = (double)ldg(E + o);
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const double x = (rd(ce[i] + q) * rd(ae[i] + q)) * j;
        s1[i] += x;
        s2[i] = fma(x, e, s2[i]);
      }
    }
  }
  double* row = C.RJ + (size_t)k * C.nrseg * 2;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    stg(row + 2 * it.e[i], sl[i]);
    stg(row + 2 * it.e[i] + 1, 0.0);
  }
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    stg(row + 2 * it.e[NL + i], s1[i]);
    stg(row + 2 * it.e[NL + i] + 1, s2[i]);
  }
}

template <typename TB, bool SC>
__device__ __forceinline__ void rates_shape(const ColDev& C, const RItem& it, int k,
                                            const TB* __restrict__ VTt, const TB* __restrict__ EbfTt) {
  switch (it.nl * 8 + it.ne) {
#define RB(L, E) \
  case L * 8 + E: rates_block<TB, L, E, SC>(C, it, k, VTt, EbfTt); break;
    RB(0, 1) RB(0, 2) RB(0, 3) RB(0, 4)
    RB(1, 0) RB(1, 1) RB(1, 2) RB(1, 3) RB(1, 4)
    RB(2, 0) RB(2, 1) RB(2, 2) RB(2, 3) RB(2, 4)
    RB(3, 0) RB(3, 1) RB(3, 2) RB(3, 3) RB(3, 4)
    RB(4, 0) RB(4, 1) RB(4, 2) RB(4, 3) RB(4, 4)
#undef RB
    default: break;
  }
}

// The column state and the block descriptor are read with independent
// scalar loads, so that a wave waits for one memory round trip, not three,
// before its first table loads.  The tables follow the evaluation's
// precision, so that an FP32-form column after its FP64 fallback evaluates
// the same F as an FP64 column.
template <bool SC>
__device__ __forceinline__ void rates_item(const ColDev& C, int b, int k0, int only_mode) {
  const int mode = ldc(&C.st->mode), prec = ldc(&C.st->cur_prec);
  const RItem it = ldc_rec(C.ritem + b);
  // (velocity-field columns list edges only: their line rates come from the
  // formal-solution kernel)
  if (mode == kModeIdle || (only_mode >= 0 && mode != only_mode)) return;
  const int k = k0 + threadIdx.x;
  if (k >= C.nz) return;
  if (prec == NLTE_FP32_FORM)
    rates_shape<float, SC>(C, it, k, C.VTf, C.EbfTf);
  else
    rates_shape<double, SC>(C, it, k, C.VT, C.EbfT);
}

// ---------------------------------------------------------------------------
// radiative part of the diagonal Jacobian blocks (Sect. 2.5.1, 2.5.2 first
// solution):  P_ij += sum_nu alpha_i (beta_j D_chi + gamma_j D_eta).
// alpha_i, beta_j and gamma_j are sums over the transitions touching a level,
// so the block is a sum over pairs of transitions (t, t') of
//   M1 = sum_nu cw_t A_t V_t' D_chi,
//   M2 = sum_nu cw_t A_t g_t' V_t' (2 h nu^3/c^2 D_eta - D_chi),
// over the intersection of their windows, A_t = V_t (n_l - g_t n_u); the
// assembly scatters M1, M2 to the levels.
//
// The sums run per piece of the frequency axis on which the covering set of
// transitions is constant, in blocks of NT x NU pairs: per frequency a lane
// (one depth) loads D_chi, D_eta, e^{-h nu/kT} and the V of the block's
// transitions once and updates all NT x NU pairs, instead of reloading them
// for every pair.  SAME: the two transition lists are the same (NT == NU).
// ---------------------------------------------------------------------------
struct PairSide {
  const double* V;  // V at the piece's first frequency, this lane's depth
  int vs;           // step per frequency (nz for line tables, 1 for edges)
  double g0, gE;    // g = g0 + gE e^{-h nu/kT} (lines: g0 = g_l/g_u; edges: gE = n*_l/n*_c)
};

__device__ __forceinline__ PairSide pair_side(const ColDev& C, int t, int f0, int k) {
  const TrDev& T = C.tr[t];
  const int wlo = uni(T.wlo), voff = uni(T.voff);
  PairSide S;
  if (t < C.nline) {
    S.V = C.VT + voff + (size_t)(f0 - wlo) * C.nz + k;
    S.vs = C.nz;
    S.g0 = uni(T.g);
    S.gE = 0.0;
  } else {
    S.V = C.V + voff + (f0 - wlo);
    S.vs = 1;
    S.g0 = 0.0;
    S.gE = C.rho_bf[k * C.nbf + (t - C.nline)];
  }
  return S;
}

template <int NT, int NU, bool SAME>
__device__ __forceinline__ void pair_block(const ColDev& C, const PItem& it, int k) {
  const int nz = C.nz, L = C.L, f0 = it.f0, nf = it.f1 - it.f0;
  PairSide ts[NT], us[NU];
  const double* cw[NT];
  double pa[NT], pb[NT];  // n_l - g n_u = pa - pb e^{-h nu/kT}
  bool edge = false;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const int t = it.t[i];
    const TrDev& T = C.tr[t];
    ts[i] = pair_side(C, t, f0, k);
    cw[i] = C.cw + uni(T.cwoff) + (f0 - uni(T.wlo));
    const double nl = C.eval_n[k * L + uni(T.lo)], nu = C.eval_n[k * L + uni(T.up)];
    pa[i] = nl - ts[i].g0 * nu;
    pb[i] = ts[i].gE * nu;
    edge |= t >= C.nline;
  }
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const int u = it.u[j];
    us[j] = SAME ? ts[j] : pair_side(C, u, f0, k);
    edge |= u >= C.nline;
  }
  const int zp = C.zp;  // rows of the derivatives and of e^{-h nu/kT}
  const double* DX = C.DchiT + (size_t)f0 * zp + k;
  const double* DE = C.DetaT + (size_t)f0 * zp + k;
  const double* EB = edge ? C.EbfT + (size_t)f0 * zp + k : DX;  // DX: any valid address
  const double* gam = C.gam + f0;
  double m1[NT][NU], m2[NT][NU];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NU; ++j) m1[i][j] = m2[i][j] = 0.0;
  for (int q = 0; q < nf; ++q) {
    const size_t o = (size_t)q * zp;
    const double dx = ldg(DX + o), de = ldg(DE + o);
    const double E = edge ? ldg(EB + o) : 0.0;
    const double dd = ldc(gam + q) * de - dx;  // per-frequency operands: scalar loads
    double vt[NT], a[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      vt[i] = ldg(ts[i].V + (size_t)q * ts[i].vs);
      a[i] = ldc(cw[i] + q) * vt[i] * (pa[i] - pb[i] * E);
    }
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double v = SAME ? vt[j] : ldg(us[j].V + (size_t)q * us[j].vs);
      const double b = v * dx, c = (us[j].g0 + us[j].gE * E) * v * dd;
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        m1[i][j] = fma(a[i], b, m1[i][j]);
        m2[i][j] = fma(a[i], c, m2[i][j]);
      }
    }
  }
  // M is [entry][nz][2]: lanes (depths) store contiguously
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      double* dst = C.M + ((size_t)(it.e0 + i * it.es + j) * nz + k) * 2;
      stg(dst, m1[i][j]);
      stg(dst + 1, m2[i][j]);
    }
}

__device__ __forceinline__ void pair_item(const ColDev& C, int p, int k0) {
  // state and block descriptor: independent scalar loads
  const int mode = ldc(&C.st->mode);
  const PItem it = ldc_rec(C.pitem + p);
  if (mode != kModeNewton || C.vel) return;  // velocity-field columns: k_pairsum_vel
  const int k = k0 + threadIdx.x;
  if (k >= C.nz) return;
  const int shape = (it.same ? 16 : 0) + (it.nt - 1) * 4 + (it.nu - 1);
  switch (shape) {
#define PB(NT, NU) \
    case (NT - 1) * 4 + (NU - 1): pair_block<NT, NU, false>(C, it, k); break;
    PB(1, 1) PB(1, 2) PB(1, 3) PB(1, 4) PB(2, 1) PB(2, 2) PB(2, 3) PB(2, 4)
    PB(3, 1) PB(3, 2) PB(3, 3) PB(3, 4) PB(4, 1) PB(4, 2) PB(4, 3) PB(4, 4)
#undef PB
    case 16 + 0: pair_block<1, 1, true>(C, it, k); break;
    case 16 + 5: pair_block<2, 2, true>(C, it, k); break;
    case 16 + 10: pair_block<3, 3, true>(C, it, k); break;
    case 16 + 15: pair_block<4, 4, true>(C, it, k); break;
    default: break;
  }
}

// Rate integrals of a step: one item per (column, rate block of a piece, 64
// depths), lane per depth; only_mode >= 0: the columns in that mode only.
template <bool SC>
__global__ __launch_bounds__(64) void k_depthwork(const ColDev* __restrict__ cols,
                                                  const int4* __restrict__ work, int nwork,
                                                  int only_mode) {
  // the items of a column are consecutive in the list: keeping them on one
  // XCD lets its transitions share the column's J in that XCD's L2
  const int w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= nwork) return;
  const int4 it = work[w];
  const int col = uni(it.x), idx = uni(it.y), k0 = uni(it.z);
  rates_item<SC>(cols[col], idx, k0, only_mode);
}

// Launches of at least this many rate items (8 waves per CU) read the
// per-frequency rate data with scalar loads; smaller ones with vector loads.
// Measured on the 4096-column batch and on one 256-depth column: scalar
// loads take the batch's F-only residual from 4.76 to 4.55 ms and slow the
// single column's from 0.441 to 0.463 ms (the same F either way).
constexpr int kRateScalarMin = 2048;

static void launch_depthwork(const BatchWork& bw, size_t lds, hipStream_t s, int only_mode) {
  if (bw.nrate0 >= kRateScalarMin)
    k_depthwork<true><<<bw.nrate0, 64, lds, s>>>(bw.cols, bw.rate_work, bw.nrate0, only_mode);
  else
    k_depthwork<false><<<bw.nrate0, 64, lds, s>>>(bw.cols, bw.rate_work, bw.nrate0, only_mode);
}

// Preconditioner pair sums of the columns in Newton mode: one item per
// (column, pair-sum block, 64 depths), lane per depth.  A kernel of its own:
// the block's accumulators need about three times the registers of the rate
// integrals, which would otherwise run at the lower occupancy too.
__global__ __launch_bounds__(64) void k_pairsum(const ColDev* __restrict__ cols,
                                                const int4* __restrict__ work, int nwork) {
  const int w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= nwork) return;
  const int4 it = work[w];
  const int col = uni(it.x), idx = uni(it.y), k0 = uni(it.z);
  pair_item(cols[col], idx, k0);
}

// ---------------------------------------------------------------------------
// assembly: rates, F rows, conservation rows, rho, preconditioner blocks
// ---------------------------------------------------------------------------
// One workgroup per kAsmDepths depths of a column.  Phase 1 spreads the
// (depth, transition) pairs over all threads: the segment sums are added up,
// the rates and total rates written out and each transition's net and gross
// flows parked in LDS.  Phase 2 gives each depth one thread, which adds the
// flows to the levels in transition order (the order fixes the rounding of F),
// and phase 3 sets the conservation row and writes F, G and the per-depth
// scaled residual.  Transitions go through LDS kAsmTr at a time.
constexpr int kAsmThreads = 256;
constexpr int kAsmDepths = 16;
constexpr int kAsmTr = 64;

__global__ __launch_bounds__(kAsmThreads) void k_assemble(const ColDev* __restrict__ cols,
                                                          const int* __restrict__ act, int nsub) {
  __shared__ double sK[kAsmDepths][kAsmTr + 1], sX[kAsmDepths][kAsmTr + 1];
  __shared__ double sF[kAsmDepths][kMaxLev + 1], sG[kAsmDepths][kMaxLev + 1];
  const int ci = blockIdx.x / nsub, sub = blockIdx.x - ci * nsub;
  const ColDev& C = cols[act ? act[ci] : ci];
  const int mode = uni(C.st->mode);
  if (mode == kModeIdle) return;
  const int nz = C.nz, L = C.L, ntr = C.ntr, nline = C.nline, nrseg = C.nrseg;
  const int k0 = sub * kAsmDepths;
  if (k0 >= nz) return;
  const int nd = min(kAsmDepths, nz - k0);
  const int tx = threadIdx.x;
  const double* __restrict__ en = C.eval_n;
  if (tx < nd)
    for (int i = 0; i < L; ++i) {
      sF[tx][i] = 0.0;
      sG[tx][i] = 0.0;
    }
  for (int t0 = 0; t0 < ntr; t0 += kAsmTr) {
    const int nt = min(kAsmTr, ntr - t0);
    for (int id = tx; id < nd * nt; id += kAsmThreads) {
      const int kk = id / nt, tt = id - kk * nt;
      const int k = k0 + kk, t = t0 + tt;
      const TrDev& T = C.tr[t];
      const double* __restrict__ rj = C.RJ + ((size_t)k * nrseg + T.sfirst) * 2;
      // the transition's pieces, added in frequency order (positive terms,
      // a few dozen at most: plain sums stay within 1e-14 relative)
      const int ns = T.nseg;
      double Rlu = ldg(rj), Rx = ldg(rj + 1);
      for (int q = 1; q < ns; ++q) {
        Rlu += ldg(rj + 2 * q);
        Rx += ldg(rj + 2 * q + 1);
      }
      const size_t kt = (size_t)k * ntr + t;
      const double Rsp = ldg(C.Rsp + kt);
      const double Rul = (t < nline) ? T.g * (Rsp + Rlu)
                                     : ldg(C.rho_bf + (size_t)k * C.nbf + (t - nline)) * (Rsp + Rx);
      stg(C.R + 2 * kt, Rlu);
      stg(C.R + 2 * kt + 1, Rul);
      const double up_rate = ldg(C.C_lu + kt) + Rlu;
      const double dn_rate = ldg(C.C_ul + kt) + Rul;
      stg(C.Rtot + 2 * kt, up_rate);
      stg(C.Rtot + 2 * kt + 1, dn_rate);
      const double out_l = ldg(en + (size_t)k * L + T.lo) * up_rate;
      const double out_u = ldg(en + (size_t)k * L + T.up) * dn_rate;
      sK[kk][tt] = out_l - out_u;
      sX[kk][tt] = fabs(out_l) + fabs(out_u);
    }
    __syncthreads();
    if (tx < nd) {
      double* Fk = sF[tx];
      double* Gk = sG[tx];
      for (int tt = 0; tt < nt; ++tt) {
        const TrDev& T = C.tr[t0 + tt];
        const int lo = uni(T.lo), up = uni(T.up);
        const double kap = sK[tx][tt], gross = sX[tx][tt];
        Fk[lo] += kap;
        Fk[up] -= kap;
        Gk[lo] += gross;
        Gk[up] += gross;
      }
    }
    __syncthreads();
  }
  if (tx >= nd) return;
  const int k = k0 + tx;
  const double* nk = en + (size_t)k * L;
  double* Fk = sF[tx];
  double* Gk = sG[tx];
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
}

// Preconditioner blocks of Newton-mode columns: one thread per (entry,
// depth) gathers its contributions (Gamma from the total rates, the
// radiative part from the pair sums) from a per-column list, then the
// conservation row of the depth becomes -1 (the original row is kept in
// Psave).  Threads are numbered depth-fastest, so a wave walks one entry's
// list in step and reads the pair sums of consecutive depths together.
__global__ __launch_bounds__(256) void k_pblock(const ColDev* __restrict__ cols,
                                                const int2* __restrict__ work, int nwork) {
  const int w = blockIdx.x;
  if (w >= nwork) return;
  const int col = uni(work[w].x), base = uni(work[w].y);
  const ColDev& C = cols[col];
  if (uni(C.st->mode) != kModeNewton) return;
  const int L = C.L, LL = L * L, nz = C.nz;
  const int id = base + threadIdx.x;
  if (id >= nz * LL) return;
  const int ij = id / nz, k = id - ij * nz;
  const int i = ij / L, j = ij - i * L;
  const double* Rt = C.Rtot + (size_t)k * C.ntr * 2;
  const double* Mk = C.M + (size_t)k * 2;
  const size_t ms = (size_t)C.nz * 2;
  double s = 0.0;
  for (int e = C.pg_ptr[ij]; e < C.pg_ptr[ij + 1]; ++e) {
    const int code = C.pg_code[e];
    const int kind = (code >> 1) & 3, idx = code >> 3;
    const double v = kind < 2 ? Rt[idx * 2 + kind] : Mk[idx * ms + (kind - 2)];
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
template <typename R>
static void launch_opacity(int kg, int ntiles, int maxnz, hipStream_t s, const ColDev* cols,
                           const Tile* tiles) {
  // about 4096 waves in all, at most one per depth group
  const int ngrp = (maxnz + kg - 1) / kg;
  const int nsplit = std::max(1, std::min(ngrp, 4096 / std::max(ntiles, 1)));
  const int bx = (ntiles * nsplit + 3) / 4;
  switch (kg) {
    case 4: k_opacity<R, 4><<<bx, 256, 0, s>>>(cols, tiles, ntiles, nsplit); break;
    case 16: k_opacity<R, 16><<<bx, 256, 0, s>>>(cols, tiles, ntiles, nsplit); break;
    default: k_opacity<R, 8><<<bx, 256, 0, s>>>(cols, tiles, ntiles, nsplit); break;
  }
}

// Side streams of the formal-solution phase, one set per host thread and
// device (a thread's launches are ordered by its own events, so threads
// never share an event between a record and the matching wait).  Created at
// the default priority, outside any graph capture (residual_streams_init).
namespace {
struct SideStreams {
  int ready = 0;
  hipStream_t st[3];
  hipEvent_t fork, join[3];
};
thread_local SideStreams tls_side[64];
}  // namespace

static hipError_t side_streams(SideStreams** out) {
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  SideStreams& S = tls_side[d & 63];
  if (!S.ready) {
    for (int i = 0; i < 3; ++i) {
      if ((e = hipStreamCreateWithFlags(&S.st[i], hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&S.join[i], hipEventDisableTiming)) != hipSuccess) return e;
    }
    if ((e = hipEventCreateWithFlags(&S.fork, hipEventDisableTiming)) != hipSuccess) return e;
    S.ready = 1;
  }
  *out = &S;
  return hipSuccess;
}

hipError_t residual_streams_init() {
  SideStreams* S = nullptr;
  return side_streams(&S);
}

__global__ __launch_bounds__(256) void k_fill_int(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_residual(const BatchWork& bw, hipStream_t s, hipEvent_t* ev) {
  // the first failing event or stream call, else the launch status at the end
  hipError_t er = hipSuccess;
  auto chk = [&er](hipError_t x) {
    if (er == hipSuccess) er = x;
  };
  if (ev) chk(hipEventRecord(ev[0], s));
  const int nblk = bw.act ? bw.nact : bw.ncol;
  const bool mlists = bw.mlist && bw.mcount && bw.gidx;
  ModeLists ml{};
  if (mlists) {
    ml.gidx = bw.gidx;
    ml.mlist = bw.mlist;
    ml.mcount = bw.mcount;
    ml.ntiles = bw.ntiles;
    for (int g = 0; g < bw.ngroup; ++g) {
      ml.first[g] = bw.groups[g].first;
      ml.fp32[g] = bw.groups[g].prec == NLTE_FP32_FORM;
    }
    k_fill_int<<<1, 4 * kMaxGroups, 0, s>>>(bw.mcount, 4 * kMaxGroups, 0);
  }
  k_coef<<<nblk, 256, 0, s>>>(bw.cols, bw.act, ml);
  for (int g = 0; g < bw.ngroup; ++g) {
    const TileGroup& G = bw.groups[g];
    if (G.vel) continue;  // the velocity formal solution makes its opacity itself
    const Tile* tl = bw.tiles + G.first;
    const bool fused32 = !G.scan && G.count >= kFuseMinTiles;  // made inside the formal solution
    if (G.prec == NLTE_FP32_FORM && !fused32)
      launch_opacity<float>(bw.opac_depths, G.count, bw.maxnz, s, bw.cols, tl);
    if (G.prec == NLTE_FP64 || bw.fallback)
      launch_opacity<double>(bw.opac_depths, G.count, bw.maxnz, s, bw.cols, tl);
  }
  // Formal solutions: the F-mode launch of each group in its own precision
  // on s, the Newton-mode launches and the FP64 launches of FP32-form groups
  // (fallback columns) on side streams.  The launches of a residual call
  // touch disjoint columns (each checks its columns' mode and precision), so
  // they may overlap: late in a batch most of them cover a few columns each
  // and would otherwise queue up their depth-recursion latencies.
  SideStreams* SS = nullptr;
  if (!bw.single_stream) {
    const hipError_t e = side_streams(&SS);
    if (e != hipSuccess) return e;
  }
  if (ev) chk(hipEventRecord(ev[1], s));
  if (SS) {
    chk(hipEventRecord(SS->fork, s));
    for (int i = 0; i < 3; ++i) chk(hipStreamWaitEvent(SS->st[i], SS->fork, 0));
  }
  const hipStream_t sNewton = SS ? SS->st[0] : s, sF64 = SS ? SS->st[1] : s, sN64 = SS ? SS->st[2] : s;
  for (int g = 0; g < bw.ngroup; ++g) {
    const TileGroup& G = bw.groups[g];
    const int nb = bw.formal_wpb;
    const Tile* tl = bw.tiles + G.first;
    const int fused = G.count >= kFuseMinTiles;  // FP32 recursion only
    const bool f32 = G.prec == NLTE_FP32_FORM;
    // FP64 launches: on s / sNewton for FP64 groups, on sF64 / sN64 for the
    // fallback columns of FP32-form groups
    const hipStream_t dF = f32 ? sF64 : s, dN = f32 ? sN64 : sNewton;
    // this step's lists (sequential groups): [0] F, [1] Newton in the group's
    // precision, [2] F, [3] Newton in FP64 for an FP32-form group's fallback
    // columns
    const bool gl = mlists && !G.scan;
    auto lst = [&](int li) -> const Tile* {
      return gl ? bw.mlist + (size_t)li * bw.ntiles + G.first : nullptr;
    };
    auto cnt = [&](int li) -> const int* { return gl ? bw.mcount + 4 * g + li : nullptr; };
    const int o64 = f32 ? 2 : 0;
    if (G.vel) {  // nlte_velocity.hip; streams as for the other groups
      if (f32) {
        launch_formal_vel(true, false, G.nmu, nb, s, bw.cols, tl, G.count, lst(0), cnt(0));
        if (bw.any_newton)
          launch_formal_vel(true, true, G.nmu, nb, sNewton, bw.cols, tl, G.count, lst(1), cnt(1));
      }
      if (!f32 || bw.fallback) {
        launch_formal_vel(false, false, G.nmu, nb, dF, bw.cols, tl, G.count, lst(o64), cnt(o64));
        if (bw.any_newton)
          launch_formal_vel(false, true, G.nmu, nb, dN, bw.cols, tl, G.count, lst(o64 + 1),
                            cnt(o64 + 1));
      }
      continue;
    }
    if (G.scan) {
      if (f32) {
        launch_formal_scan_mu<float, false>(G.nmu, s, bw.cols, tl, G.count);
        if (bw.any_newton) launch_formal_scan_mu<float, true>(G.nmu, sNewton, bw.cols, tl, G.count);
      }
      if (!f32 || bw.fallback) {
        launch_formal_scan_mu<double, false>(G.nmu, dF, bw.cols, tl, G.count);
        if (bw.any_newton) launch_formal_scan_mu<double, true>(G.nmu, dN, bw.cols, tl, G.count);
      }
      continue;
    }
    if (f32) {
      launch_formal_mu<float, false>(G.nmu, nb, s, bw.cols, tl, G.count, fused, lst(0), cnt(0));
      if (bw.any_newton)
        launch_formal_mu<float, true>(G.nmu, nb, sNewton, bw.cols, tl, G.count, fused, lst(1), cnt(1));
    }
    if (!f32 || bw.fallback) {
      launch_formal_mu<double, false>(G.nmu, nb, dF, bw.cols, tl, G.count, 0, lst(o64), cnt(o64));
      if (bw.any_newton)
        launch_formal_mu<double, true>(G.nmu, nb, dN, bw.cols, tl, G.count, 0, lst(o64 + 1),
                                       cnt(o64 + 1));
    }
  }
  if (ev) chk(hipEventRecord(ev[6], s));  // end of the F-mode launches on s
  // The rate integrals stream V and J of many (column, segment) pairs at
  // once; at full occupancy (32 waves per CU) they ran 20 % slower than with
  // at most 13.  The kernel uses no LDS: the allocation only caps waves per CU
  // (160 KB / 12 KB).
  constexpr size_t kDepthworkLds = 12 * 1024;
  bool any_vel = false;
  for (int g = 0; g < bw.ngroup; ++g) any_vel |= bw.groups[g].vel != 0;
  const bool pairs = bw.any_newton && bw.nrate > bw.nrate0;
  if (SS) {
    // The F-mode columns' rate integrals start once their formal solutions
    // are done (s, and sF64 for fallback columns), while the Newton-mode
    // launches (longer: derivatives) may still run; the Newton-mode columns'
    // rate integrals and pair sums follow their own formal solutions on
    // sNewton.  Items of columns in the other mode return at once.
    chk(hipEventRecord(SS->join[1], SS->st[1]));
    chk(hipStreamWaitEvent(s, SS->join[1], 0));
    if (ev) chk(hipEventRecord(ev[2], s));
    if (bw.nrate0 > 0)
      launch_depthwork(bw, kDepthworkLds, s, kModeF);
    if (bw.any_newton) {
      chk(hipEventRecord(SS->join[2], SS->st[2]));
      chk(hipStreamWaitEvent(sNewton, SS->join[2], 0));
      if (bw.nrate0 > 0)
        launch_depthwork(bw, 0, sNewton, kModeNewton);
      if (pairs)
        k_pairsum<<<bw.nrate - bw.nrate0, 64, 0, sNewton>>>(bw.cols, bw.rate_work + bw.nrate0,
                                                             bw.nrate - bw.nrate0);
      if (any_vel && pairs)
        launch_pairsum_vel(bw.cols, bw.rate_work + bw.nrate0, bw.nrate - bw.nrate0, sNewton);
    }
    for (int i = 0; i < 3; i += 2) {
      chk(hipEventRecord(SS->join[i], SS->st[i]));
      chk(hipStreamWaitEvent(s, SS->join[i], 0));
    }
  } else {
    if (ev) chk(hipEventRecord(ev[2], s));
    if (bw.nrate0 > 0)
      launch_depthwork(bw, kDepthworkLds, s, -1);
    if (pairs)
      k_pairsum<<<bw.nrate - bw.nrate0, 64, 0, s>>>(bw.cols, bw.rate_work + bw.nrate0,
                                                     bw.nrate - bw.nrate0);
    if (any_vel && pairs)
      launch_pairsum_vel(bw.cols, bw.rate_work + bw.nrate0, bw.nrate - bw.nrate0, s);
  }
  if (ev) chk(hipEventRecord(ev[3], s));
  {
    const int nsub = (bw.maxnz + kAsmDepths - 1) / kAsmDepths;
    k_assemble<<<nblk * nsub, kAsmThreads, 0, s>>>(bw.cols, bw.act, nsub);
  }
  if (bw.any_newton && bw.npb > 0) k_pblock<<<bw.npb, 256, 0, s>>>(bw.cols, bw.pb_work, bw.npb);
  if (bw.any_tangent) chk(launch_tangent(bw, s));
  if (ev) chk(hipEventRecord(ev[4], s));
  if (er != hipSuccess) return er;
  return hipGetLastError();
}

// Work lists of a batch (host side): formal-solution tiles, rate items and
// preconditioner items for every column.  Returns the number of rate items,
// which come first in `rate`; the pair-sum blocks follow.
int build_work_lists(const ColDev* hc, int ncol, std::vector<Tile>& tiles,
                      std::vector<TileGroup>& groups, std::vector<int4>& rate,
                      std::vector<int2>& pblock, int& maxL, const int* sel, int nsel) {
  // sel: the columns to list (indices into hc), or NULL for all of them
  std::vector<int> all;
  if (!sel) {
    all.resize(ncol);
    for (int c = 0; c < ncol; ++c) all[c] = c;
    sel = all.data();
    nsel = ncol;
  }
  // formal-solution tiles grouped by (variant, precision, angle count); the
  // velocity-field columns (sequential) by (precision, angle count)
  for (int scan = 0; scan < 2; ++scan)
    for (int prec = 0; prec < 2; ++prec)
      for (int nmu = 1; nmu <= kMaxMu; ++nmu) {
        TileGroup G{prec, nmu, (int)tiles.size(), 0, scan, 0};
        for (int q = 0; q < nsel; ++q) {
          const int c = sel[q];
          if (hc[c].prec == prec && hc[c].nmu == nmu && hc[c].scan == scan && !hc[c].vel)
            for (int ch = 0; ch < hc[c].nchunk; ++ch) tiles.push_back(Tile{c, ch});
        }
        G.count = (int)tiles.size() - G.first;
        if (G.count) groups.push_back(G);
      }
  for (int prec = 0; prec < 2; ++prec)
    for (int nmu = 1; nmu <= kMaxMu; ++nmu) {
      TileGroup G{prec, nmu, (int)tiles.size(), 0, 0, 1};
      for (int q = 0; q < nsel; ++q) {
        const int c = sel[q];
        if (hc[c].vel && hc[c].prec == prec && hc[c].nmu == nmu)
          for (int ch = 0; ch < hc[c].nchunk; ++ch) tiles.push_back(Tile{c, ch});
      }
      G.count = (int)tiles.size() - G.first;
      if (G.count) groups.push_back(G);
    }
  // rate items (kind 0), then preconditioner pair-sum blocks (kind 1), each
  // kind column by column
  maxL = 0;
  for (int q = 0; q < nsel; ++q) {
    const int c = sel[q];
    for (int b = 0; b < hc[c].nz * hc[c].L * hc[c].L; b += 256) pblock.push_back(make_int2(c, b));
  }
  for (int q = 0; q < nsel; ++q) {
    const int c = sel[q];
    const ColDev& C = hc[c];
    maxL = std::max(maxL, C.L);
    for (int b = 0; b < C.nritem; ++b)
      for (int k0 = 0; k0 < C.nz; k0 += kWave) rate.push_back(make_int4(c, b, k0, 0));
  }
  const int nrate0 = (int)rate.size();
  for (int q = 0; q < nsel; ++q) {
    const ColDev& C = hc[sel[q]];
    for (int p = 0; p < C.npitem; ++p)
      for (int k0 = 0; k0 < C.nz; k0 += kWave) rate.push_back(make_int4(sel[q], p, k0, 1));
  }
  return nrate0;
}

}  // namespace nlte
