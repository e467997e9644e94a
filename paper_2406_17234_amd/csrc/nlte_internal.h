// Internal layout of a column on the device and helpers shared by the
// library's HIP translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

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
constexpr int kScanThreads = 256;  // depths of a column with the depth-parallel formal solution

// Loads and stores through the global address space (the pointers live in
// column descriptors, so the compiler cannot infer it and would emit flat
// accesses).
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void stg(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// Wave-uniform loads of data no kernel writes while it runs (populations of
// the evaluation, per-depth tables): through the constant address space, so
// they use the scalar data cache.
template <typename T>
__device__ __forceinline__ T ldc(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

// The same for a small record of ints (copied int by int; the compiler
// merges the loads into a few wide scalar loads).
template <typename T>
__device__ __forceinline__ T ldc_rec(const T* p) {
  static_assert(sizeof(T) % sizeof(int) == 0, "record of ints");
  T v;
  int* d = reinterpret_cast<int*>(&v);
  const int* s = reinterpret_cast<const int*>(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / sizeof(int)); ++i) d[i] = ldc(s + i);
  return v;
}

// Values the compiler cannot prove wave-uniform, moved to scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Work item of block b of an nb-block launch when consecutive items should
// share an XCD's L2: the blocks of a launch are dealt round-robin over the 8
// XCDs (block b runs on XCD b % 8), so the items are numbered XCD by XCD.
__device__ __forceinline__ int xcd_item(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, r = nb % kXcd;
  const int x = b % kXcd, l = b / kXcd;
  return x * q + (x < r ? x : r) + l;
}

// The same numbering when only the first nlive of a grid's items have work
// (a count known on the device only): block b gets item xcd_item(b, nlive),
// or -1 if it has none.  The blocks given an item are exactly those that
// xcd_item(., nlive) would use, all below any grid of at least nlive blocks.
__device__ __forceinline__ int xcd_live_item(int b, int nlive) {
  constexpr int kXcd = 8;
  const int q = nlive / kXcd, r = nlive % kXcd;
  const int x = b % kXcd, l = b / kXcd;
  if (l >= q + (x < r ? 1 : 0)) return -1;
  return x * q + (x < r ? x : r) + l;
}

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
  int sfirst, nseg; // its rate entries (one per piece of its window)
  double g;         // lines: g_l / g_u
  double Blu;       // lines: Einstein B_lu (for the profile-averaged intensity)
};

// Small per-column state shared by the residual kernels and the solver.
struct ColState {
  int mode;         // EvalMode of the pending evaluation
  int want_J;       // write J of the evaluation to Jeval
  int rows_own;     // kModeF: 1 = rows from the evaluated n, 0 = rows_frozen
  int jdag_fresh;   // J-dagger already refreshed at the current Newton point
  int phase;        // solver phase (see nlte_solver.hip)
  int status;       // nlte_status of the solve
  int newton_it, krylov_j, krylov_total, f_calls, stalls, ls_try, restarts, precond_calls;
  double rho_cur;   // max scaled residual at the Newton iterate
  double beta0;     // preconditioned residual norm at the start of the Newton step
  double eps_fd;    // difference step of the pending product
  double alpha;     // line-search factor
  double dn_inf;    // last population change norm
  double phi0;      // ||D^-1 P^-1 F|| at the iterate (line-search reference)
  double ftol, rtol, eps_mach, eps_scale;
  int maxiter, max_krylov, restart, max_halvings;
  int init_kind, done_flag;
  int krylov_step;  // Krylov iterations of the current Newton step
  int max_krylov_total;  // 0: no limit
  int cur_prec;     // precision the next evaluation runs in (FP32-form columns may switch to FP64)
  int fp64_fallback;  // FP32-form columns not converged after this many Newton iterations switch (0: never)
  int fp64_evals;   // FP64 evaluations after a switch
  int method;       // nlte_krylov of the solve
  int jv;           // nlte_jv of the solve
  int tan_pending;  // a tangent product (n in n, direction in eval_n) is pending
  int krylov_x0;    // initial guess of the Krylov solves: 0 zero, 1 -P^-1 F (scaled: b)
  double bi_rho, bi_alpha;  // BiCGSTAB: (r^, r) and the step of the pending half
};

// Preconditioner pair sums.  The frequency axis of a column is cut at every
// window edge (and into pieces of at most the segment length), so that on a
// piece [f0, f1) the set of transitions whose windows cover it is constant.
// A piece with s transitions has s^2 entries (t, t') in M and is summed in
// blocks of at most kPairBlk x kPairBlk of them: block entry (i, j) pairs
// transitions t[i] and u[j] and is entry e0 + i * es + j.
constexpr int kPairBlk = 4;

// Rate integrals run over the same pieces as the pair sums (the line rates
// of velocity-field columns instead come from their formal-solution kernel,
// one entry per (line, 64-frequency chunk) of its window).  One block of a
// piece: frequencies [f0, f1), nl lines t[0..nl) and ne edges t[nl..nl+ne)
// among the transitions covering it (at most kRateBlk of each); the partial
// sums of t[i] go to rate entry e[i].  A transition's entries are numbered
// in frequency order (TrDev::sfirst, nseg), and the assembly adds them in
// that order.
constexpr int kRateBlk = 4;
struct RItem {
  int f0, f1, nl, ne;
  int t[2 * kRateBlk], e[2 * kRateBlk];
};
struct PItem {
  int f0, f1, nt, nu;
  int e0, es, same, pad;  // same: u[] lists the same transitions as t[]
  int t[kPairBlk], u[kPairBlk];
};

struct ColDev {
  int nz, L, ntr, nline, nbf, nnu, nmu, prec;
  int fp;                          // row pitch of the [nz][nnu] formal-solution scratch and
                                   // FP32 tables: nnu rounded up to a multiple of 64, so that
                                   // a chunk's 64 frequencies start on a cache-line boundary
  int zp;                          // row pitch of the depth-contiguous [nnu][nz] arrays (J, the
                                   // derivatives, e^{-h nu/kT}): nz rounded up to a multiple
                                   // of 16, so that a wave's 64 depths start on a line boundary
  int nchunk, has_sca, N;          // N = nz * L
  int bg_eta;                      // 1: the caller gave the background emissivity eta_c
  int npitem, nment;               // pair-sum blocks, entries of M
  int scan;                        // 1: depth-parallel formal solution (nz <= 256)
  int nrseg, nritem;               // rate-integral entries (partial sums) and blocks
  int vel;                         // 1: velocity field, line opacity per ray (sequential)
  int nray;                        // 2 nmu: rays 0..nmu-1 outgoing, nmu..2nmu-1 ingoing
  // angles (inline: at most kMaxMu)
  double wm2[kMaxMu];     // w_m / 2
  double inv2mu[kMaxMu];  // 1 / (2 mu_m)
  float wm2f[kMaxMu], inv2muf[kMaxMu];  // the same, FP32 form
  // atmosphere
  const double *z, *dz, *T, *ne, *ntot, *chi_c, *chi_sca;
  // frequency grid and per-(k, f) tables [nz][nnu]
  const double *nu, *gam;          // gam = 2 h nu^3 / c^2
  const double *Bnu, *Ebf;         // Planck function, exp(-h nu / kT)
  const double *EC;                // thermal background emission table: Bnu (emissivity
                                   // chi_c B_nu, bg_eta = 0) or the caller's eta_c (bg_eta = 1)
  const double *EbfT;              // [nnu][zp] exp(-h nu / kT), depth-contiguous
  // transitions
  const TrDev *tr;
  const double *V;                 // per-transition V tables
  const double *VT;                // line V tables depth-contiguous ([wlen][nz] at the same offsets)
  const double *cw;                // per-transition rate weights
  const double *rho_bf;            // [nz][nbf] n*_l / n*_c
  const double *Rsp;               // [nz][ntr] n-independent part of R_ul
  const double *C_lu, *C_ul;       // [nz][ntr]
  const double *nstar;             // [nz][L]
  // velocity fields: line V tables of every ray, [nray][nz][wlen] per line at
  // offset nray * voff (the line tables come first, so the offsets are those
  // of V scaled by nray), their depth-contiguous copies VRT ([nray][wlen][nz]
  // at the same offsets); vlos [nz]
  const double *VR, *VRT, *vlos;
  // FP32 copies of V, Bnu and Ebf read by the FP32-form opacity kernel (NULL
  // for FP64 columns); n-independent, so their rounding adds no noise to F
  const float *Vf, *Bnuf, *Ebff;
  const float *ECf;                // FP32 copy of EC (rows of fp)
  const float *VTf, *EbfTf;        // FP32 copies of VT and EbfT (rate integrals; EbfTf [nnu][zp])
  // chunk -> overlapping line windows and edge windows; overlapping transition pairs
  const int *ch_lptr, *ch_line;
  const int *ch_eptr, *ch_edge;
  const RItem *ritem;              // rate-integral blocks
  const PItem *pitem;              // blocks of the preconditioner pair sums
  const int *pg_ptr, *pg_code;     // per block entry (i, j): contributions, see k_pblock
  // evaluation buffers
  ColState *st;
  double *eval_n;                  // [nz][L] populations to evaluate F at
  double *coef;                    // [ntr + 2][nz][2] level coefficients of eval_n
  double *F, *G;                   // [nz][L] residual and gross rates
  double *Jdag;                    // [nz][nnu] lagged mean intensity
  double *JT;                      // [nnu][zp] J of the last evaluation (depth-contiguous)
  // scratch of the formal solution, in the column's formal-solution precision
  // (buffers sized for doubles):
  double *Jm;                      // [nz][nnu] ingoing-ray part of J (recursion precision)
  double *XS;                      // [nz][nnu][2] chi and S of the first sweep
  double *Dchi, *Deta;             // [nz][nnu] ingoing-ray intensity derivatives
  double *DchiT, *DetaT;           // [nnu][zp] angle-averaged local intensity derivatives
  double *RJ;                      // [nz][nrseg][2] rate integrals over J, per segment
  double *M;                       // [nment][nz][2] pair sums of the radiative blocks
  double *DXR, *DER;               // velocity fields: [nray][nnu][zp] local intensity derivatives
  double *P;                       // [nz][L][L] preconditioner blocks of the last Newton-mode evaluation
  double *LU;                      // [nz][L][L] LU factors of the iterate's blocks
  double *Fsave, *Gsave;           // [nz] rate-row F and gross rate under each conservation row
  double *Psave;                   // [nz][L] preconditioner row under each conservation row
  double *R;                       // [nz][ntr][2] radiative rates of the last evaluation
  double *Rtot;                    // [nz][ntr][2] C_lu + R_lu, C_ul + R_ul
  double *rho_k;                   // [nz] max scaled residual per depth
  int *rows;                       // [nz] conservation rows used by the last evaluation
  int *rows_frozen;                // [nz] rows for kModeF evaluations
  int *piv;                        // [nz][L] pivots of the LU factors
  // solver buffers
  double *n;                       // [N] Newton iterate
  double *n_init;                  // [N] initial populations of the solve
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

// The tile of wave `wave` of this block in a formal-solution launch over a
// group of ntiles tiles: from the launch's per-step list when mcount is set
// (its first *mcount entries, dealt over the XCDs as a full grid would be),
// else the group's own list.  The chunks of a column are consecutive either
// way, so they run on one XCD and share its L2.  False: no tile.
__device__ __forceinline__ bool pick_tile(const Tile* __restrict__ tiles, int ntiles,
                                          const Tile* __restrict__ mlist,
                                          const int* __restrict__ mcount, int wave, Tile& t) {
  const int wpb = blockDim.x >> 6;
  int tid;
  if (mcount) {
    const int n = __builtin_amdgcn_readfirstlane(ldc(mcount));
    const int blk = xcd_live_item(blockIdx.x, (n + wpb - 1) / wpb);
    if (blk < 0) return false;
    tid = blk * wpb + wave;
    if (tid >= n) return false;
    tiles = mlist;
  } else {
    tid = xcd_item(blockIdx.x, gridDim.x) * wpb + wave;
    if (tid >= ntiles) return false;
  }
  t.col = __builtin_amdgcn_readfirstlane(tiles[tid].col);
  t.chunk = __builtin_amdgcn_readfirstlane(tiles[tid].chunk);
  return true;
}


// Frequency sums over a transition's window (rate integrals, preconditioner
// pair sums) run in segments of at most this many frequencies, each summed by
// its own wave, so that the longest serial chain of a wide window stays short.
// A property of the column (not of the batch it is evaluated in): columns with
// the depth-parallel formal solution, evaluated alone or few at a time, use
// the short segments.
constexpr int kSegLen = 512;
constexpr int kSegLenScan = 128;

// Level coefficients of an evaluation (k_coef), [ntr + 2][nz][2]: per
// transition and depth two values, then two background rows.
inline __host__ __device__ int ncoef(int ntr) { return 2 * ntr + 4; }

// Tiles of one (precision, angle count) group, contiguous in the tile list.
struct TileGroup {
  int prec, nmu, first, count;
  int scan;  // columns solved by the depth-parallel formal solution
  int vel;   // columns with a velocity field (sequential)
};

// Tile groups a batch can have: one per (formal-solution variant, precision,
// angle count), plus the velocity-field columns per (precision, angle count).
constexpr int kMaxGroups = 2 * 2 * kMaxMu + 2 * kMaxMu;

// Device work lists of a batch of columns.
struct BatchWork {
  const ColDev* cols = nullptr;   // device array [ncol]
  const Tile* tiles = nullptr;    // formal-solution chunks, grouped by (precision, nmu)
  TileGroup groups[kMaxGroups];
  int ngroup = 0;
  int maxnz = 0;                  // deepest column of the batch
  int fallback = 0;               // FP32-form columns may run FP64 evaluations
  const int* act = nullptr;       // columns the lists cover (NULL: all ncol), device
  int nact = 0;
  int opac_depths = 8;            // launch shapes (tuned by residual plans): depths per
  int formal_wpb = 1;             // opacity wave (4, 8, 16); waves per formal block (1, 2, 4)
  const int4* rate_work = nullptr;  // (col, segment or block, first depth, kind)
  const int2* pb_work = nullptr;  // (col, first depth-entry index)
  int ncol = 0, ntiles = 0, nrate = 0, npb = 0;
  int nrate0 = 0;                 // rate items at the front of rate_work; pair-sum blocks follow
  int any64 = 0, any32 = 0, any_newton = 1;
  int any_tangent = 0;            // columns may request tangent products
  int single_stream = 0;          // 1: every launch on the caller's stream (no side streams
                                  // are created or used)
  // Per-step mode lists (optional; NULL: every formal-solution launch walks
  // its group's whole tile list and waves of other modes return).  At the
  // start of each residual call the tiles of the sequential groups are
  // sorted by the launch that will evaluate them (F or Newton mode, in the
  // column's current precision), so that each launch starts with the waves
  // that have work.  gidx [ncol]: each column's group if that group uses the
  // lists, else -1; mlist: 4 lists of capacity ntiles (F, Newton, and the
  // FP64 F and Newton launches of an FP32-form group's fallback columns);
  // mcount: their lengths [kMaxGroups][4], cleared by a fill kernel first.
  const int* gidx = nullptr;
  Tile* mlist = nullptr;
  int* mcount = nullptr;
};

// The host copy of gidx (per-step mode lists) for the groups in bw and their
// tile list; the caller copies it to the device.
inline void set_mode_groups(const BatchWork& bw, const std::vector<Tile>& tiles, int ncol,
                            std::vector<int>& gidx) {
  gidx.assign(ncol, -1);
  for (int g = 0; g < bw.ngroup; ++g) {
    const TileGroup& G = bw.groups[g];
    if (G.scan) continue;
    for (int t = G.first; t < G.first + G.count; ++t) gidx[tiles[t].col] = g;
  }
}

// Residual launches for a batch (level coefficients and opacity, formal
// solution of every tile, rate integrals and preconditioner pair sums,
// assembly).  ev, if not NULL, holds seven events, all recorded on s:
// [0] before the coefficients, [1] before the formal-solution launches,
// [2] after the F-mode ones (with side streams: those of the FP64 side
// stream joined; the Newton-mode stream may still run), [3] after the
// lane-per-depth work and every side stream,
// [4] after assembly, [5] left to the caller, [6] after the F-mode
// formal-solution launches that run on s itself.
hipError_t launch_residual(const BatchWork& bw, hipStream_t s, hipEvent_t* ev = nullptr);
// Velocity-field columns (nlte_velocity.hip): the formal-solution launch of
// one tile group in the FP32 form or FP64 and in F or Newton mode (each wave
// skips the columns evaluated in the other; mlist/mcount: this step's list of
// the launch, as for k_formal), and the pair sums over
// the preconditioner items of a batch (other columns' items return at once).
void launch_formal_vel(bool fp32, bool newton, int nmu, int wpb, hipStream_t s, const ColDev* cols,
                       const Tile* tiles, int ntiles, const Tile* mlist = nullptr,
                       const int* mcount = nullptr);
void launch_pairsum_vel(const ColDev* cols, const int4* work, int nwork, hipStream_t s);
// Tangent-linear products (nlte_tangent.hip) of the columns whose state has
// tan_pending set: J v into F.  launch_residual runs it when bw.any_tangent.
hipError_t launch_tangent(const BatchWork& bw, hipStream_t s);
// Creates the calling thread's side streams for the current device (done
// lazily by launch_residual; call it before capturing launches into a graph).
hipError_t residual_streams_init();

// Solver driver pieces (nlte_solver.hip) shared by the batch solve and the
// server: option checks, per-column initialisation (n0[c] NULL: LTE), one
// Newton/Krylov step of every column, and a copy of the columns' states.
nlte_status check_solve_opts(const nlte_solve_opts& o);
hipError_t solver_init(const ColDev* cols, int ncol, const double* const* n0,
                       const double* const* J0, const nlte_solve_opts& o, hipStream_t s);
hipError_t solver_step(const ColDev* cols, const int* act, int n, int* done, hipStream_t s);
hipError_t solver_gather(const ColDev* cols, int ncol, ColState* out, hipStream_t s);
bool state_done(const ColState& st);
void zero_radiation_into(const ColDev* dcol, const ColDev& hc, hipStream_t s);
void state_stats(const ColState& st, nlte_solve_stats* out);

// Copies the tile groups of build_work_lists into bw; false (bw untouched)
// if there are more than kMaxGroups of them.
inline bool set_groups(BatchWork& bw, const std::vector<TileGroup>& groups) {
  if (groups.size() > (size_t)kMaxGroups) return false;
  bw.ngroup = (int)groups.size();
  for (int g = 0; g < bw.ngroup; ++g) bw.groups[g] = groups[g];
  return true;
}

// Bytes of a server-pooled column arena for a column whose plan takes
// `plan` bytes (the arena, then the column's device descriptor).
size_t pooled_arena_bytes(size_t plan);

int build_work_lists(const ColDev* hc, int ncol, std::vector<Tile>& tiles,
                     std::vector<TileGroup>& groups, std::vector<int4>& rate,
                     std::vector<int2>& pblock, int& maxL, const int* sel = nullptr,
                     int nsel = 0);

}  // namespace nlte

struct nlte_ctx {
  int device;
  int prof_on;
  nlte_profile prof;
};
