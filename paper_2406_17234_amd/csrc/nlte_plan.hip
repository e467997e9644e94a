// Residual plans: F(n) of a fixed set of columns in shared launches, with an
// optional HIP-graph capture of the launch sequence and a launch-shape tuner.
#include <vector>

#include "nlte_internal.h"

nlte_status set_err(nlte_status st, const char* fmt, ...);

namespace nlte {
const ColDev& column_dev(const nlte_column* c);
nlte_ctx* column_ctx(const nlte_column* c);
}  // namespace nlte

using namespace nlte;

#define HIP_TRY(x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return set_err(NLTE_E_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_));       \
  } while (0)

namespace {

// n_dev[c] -> eval_n of column c; F-only evaluation with the column's own
// conservation rows and precision.
__global__ void k_plan_in(const ColDev* __restrict__ cols, const double* const* __restrict__ n) {
  const ColDev& C = cols[blockIdx.x];
  const double* src = n[blockIdx.x];
  for (int i = threadIdx.x; i < C.N; i += blockDim.x) C.eval_n[i] = src[i];
  if (threadIdx.x == 0) {
    C.st->mode = kModeF;
    C.st->rows_own = 1;
    C.st->want_J = 0;
    C.st->cur_prec = C.prec;
  }
}

__global__ void k_plan_out(const ColDev* __restrict__ cols, double* const* __restrict__ F) {
  const ColDev& C = cols[blockIdx.x];
  double* dst = F[blockIdx.x];
  for (int i = threadIdx.x; i < C.N; i += blockDim.x) dst[i] = C.F[i];
  if (threadIdx.x == 0) C.st->mode = kModeIdle;
}

}  // namespace

struct nlte_plan {
  nlte_ctx* ctx = nullptr;
  int device = 0;  // ctx->device, kept so that destruction never reads ctx
  int ncol = 0;
  ColDev* cols = nullptr;
  Tile* tiles = nullptr;
  int4* rate = nullptr;
  int2* pb = nullptr;
  const double** n = nullptr;
  double** F = nullptr;
  BatchWork bw;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  nlte_plan_info info{};

  hipError_t launch(hipStream_t s) {
    k_plan_in<<<ncol, 256, 0, s>>>(cols, n);
    hipError_t e = launch_residual(bw, s);
    if (e != hipSuccess) return e;
    k_plan_out<<<ncol, 256, 0, s>>>(cols, F);
    return hipGetLastError();
  }
  ~nlte_plan() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (cap_stream) hipStreamDestroy(cap_stream);
    if (cols) hipFree(cols);
    if (tiles) hipFree(tiles);
    if (rate) hipFree(rate);
    if (pb) hipFree(pb);
    if (n) hipFree(n);
    if (F) hipFree(F);
  }
};

static nlte_status plan_tune(nlte_plan* P, hipStream_t s) {
  const int kgs[3] = {4, 8, 16}, wps[3] = {1, 2, 4};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best = 1e300;
  int bk = 8, bw = 4;
  nlte_status st = NLTE_OK;
  for (int a = 0; a < 3 && st == NLTE_OK; ++a)
    for (int b = 0; b < 3 && st == NLTE_OK; ++b) {
      P->bw.opac_depths = kgs[a];
      P->bw.formal_wpb = wps[b];
      hipError_t e = P->launch(s);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = P->launch(s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = set_err(NLTE_E_DEVICE, "plan tuning failed: %s", hipGetErrorString(e));
        break;
      }
      P->info.tune_ms[a * 3 + b] = ms / 3.0;
      if (ms < best) {
        best = ms;
        bk = kgs[a];
        bw = wps[b];
      }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  P->bw.opac_depths = bk;
  P->bw.formal_wpb = bw;
  return st;
}

extern "C" nlte_status nlte_plan_create(nlte_ctx* ctx, nlte_column* const* cols, int32_t ncol,
                                        const double* const* n_dev, double* const* F_dev,
                                        int32_t flags, hipStream_t s, nlte_plan** out) {
  if (!ctx || !cols || ncol <= 0 || !n_dev || !F_dev || !out)
    return set_err(NLTE_E_INVALID, "bad plan arguments");
  std::vector<ColDev> hc(ncol);
  for (int c = 0; c < ncol; ++c) {
    if (!cols[c] || !n_dev[c] || !F_dev[c]) return set_err(NLTE_E_INVALID, "NULL entry %d", c);
    if (column_ctx(cols[c]) != ctx) return set_err(NLTE_E_INVALID, "column %d from another context", c);
    for (int d = 0; d < c; ++d)
      if (cols[d] == cols[c]) return set_err(NLTE_E_INVALID, "column %d appears twice", c);
    hc[c] = column_dev(cols[c]);
  }
  HIP_TRY(hipSetDevice(ctx->device));
  nlte_plan* P = new nlte_plan();
  P->ctx = ctx;
  P->device = ctx->device;
  P->ncol = ncol;
  std::vector<Tile> tiles;
  std::vector<TileGroup> groups;
  std::vector<int4> rate;
  std::vector<int2> pb;
  int maxL = 0;
  const int nrate0 = build_work_lists(hc.data(), ncol, tiles, groups, rate, pb, maxL);
  auto fail = [&](nlte_status st) {
    delete P;
    return st;
  };
#define PLAN_TRY(x)                                                                         \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess)                                                                   \
      return fail(set_err(NLTE_E_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_)));      \
  } while (0)
  PLAN_TRY(hipMalloc(&P->cols, ncol * sizeof(ColDev)));
  PLAN_TRY(hipMalloc(&P->tiles, std::max<size_t>(1, tiles.size()) * sizeof(Tile)));
  PLAN_TRY(hipMalloc(&P->rate, std::max<size_t>(1, rate.size()) * sizeof(int4)));
  PLAN_TRY(hipMalloc(&P->pb, std::max<size_t>(1, pb.size()) * sizeof(int2)));
  PLAN_TRY(hipMalloc(&P->n, ncol * sizeof(double*)));
  PLAN_TRY(hipMalloc(&P->F, ncol * sizeof(double*)));
  PLAN_TRY(hipMemcpyAsync(P->cols, hc.data(), ncol * sizeof(ColDev), hipMemcpyHostToDevice, s));
  PLAN_TRY(hipMemcpyAsync(P->tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
  PLAN_TRY(hipMemcpyAsync(P->rate, rate.data(), rate.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  PLAN_TRY(hipMemcpyAsync(P->pb, pb.data(), pb.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  PLAN_TRY(hipMemcpyAsync(P->n, n_dev, ncol * sizeof(double*), hipMemcpyHostToDevice, s));
  PLAN_TRY(hipMemcpyAsync(P->F, F_dev, ncol * sizeof(double*), hipMemcpyHostToDevice, s));
  BatchWork& bw = P->bw;
  bw.cols = P->cols;
  bw.tiles = P->tiles;
  bw.rate_work = P->rate;
  bw.pb_work = P->pb;
  bw.ncol = ncol;
  bw.ntiles = (int)tiles.size();
  bw.nrate = (int)rate.size();
  bw.nrate0 = nrate0;
  bw.npb = (int)pb.size();
  bw.any_newton = 0;  // F only: no preconditioner work
  if (!set_groups(bw, groups)) return fail(set_err(NLTE_E_INVALID, "too many tile groups"));
  int64_t dp = 0;
  for (int c = 0; c < ncol; ++c) {
    bw.maxnz = std::max(bw.maxnz, hc[c].nz);
    if (hc[c].prec == NLTE_FP64) bw.any64 = 1; else bw.any32 = 1;
    dp += (int64_t)hc[c].nz * hc[c].nnu * 2 * hc[c].nmu;
  }
  P->info.ncol = ncol;
  P->info.depth_points = dp;
  if (flags & NLTE_PLAN_TUNE) {
    const nlte_status st = plan_tune(P, s);
    if (st != NLTE_OK) return fail(st);
  }
  P->info.opac_depths = bw.opac_depths;
  P->info.formal_wpb = bw.formal_wpb;
  if (flags & NLTE_PLAN_GRAPH) {
    // capture on a stream of the plan's own, ordered after the setup above
    PLAN_TRY(hipStreamSynchronize(s));
    PLAN_TRY(residual_streams_init());
    PLAN_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    PLAN_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipError_t le = P->launch(P->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(P->cap_stream, &g);
    P->graph = g;
    PLAN_TRY(le);
    PLAN_TRY(ce);
    PLAN_TRY(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
    P->info.graph = 1;
  }
#undef PLAN_TRY
  *out = P;
  return NLTE_OK;
}

extern "C" nlte_status nlte_plan_run(nlte_plan* P, hipStream_t s) {
  if (!P) return set_err(NLTE_E_INVALID, "NULL plan");
  HIP_TRY(hipSetDevice(P->ctx->device));
  if (P->exec) {
    HIP_TRY(hipGraphLaunch(P->exec, s));
  } else {
    HIP_TRY(P->launch(s));
  }
  return NLTE_OK;
}

extern "C" nlte_status nlte_plan_info_get(const nlte_plan* P, nlte_plan_info* out) {
  if (!P || !out) return set_err(NLTE_E_INVALID, "NULL argument");
  *out = P->info;
  return NLTE_OK;
}

extern "C" void nlte_plan_destroy(nlte_plan* P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  delete P;
}
