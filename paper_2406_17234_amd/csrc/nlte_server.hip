// Serving loop: continuous batching of JFNK column solves on one device.
//
// One host thread per server drives a non-blocking HIP stream.  Each pass of
// its loop admits queued requests (FIFO, within the HBM budget and the slot
// count), initialises their solver state on the device, replays kSteps solver
// steps over every column in flight (the same launches as the batch solve:
// one residual evaluation per column per step, then one Newton/Krylov step),
// reads back the columns' states and retires the finished ones.  Work lists
// are rebuilt whenever the set of columns in flight changes.
//
// A request is either a column the caller created (its device memory exists
// before admission and is counted while it is in flight) or a problem
// description copied at submission: its column is created (device memory
// allocated, n-independent setup run) when the request is admitted within
// the budget, and destroyed, after its populations are copied out, when it
// retires, so the budget bounds the device memory the requests hold.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nlte_internal.h"

nlte_status set_err(nlte_status st, const char* fmt, ...);

namespace nlte {
const ColDev& column_dev(const nlte_column* c);
nlte_ctx* column_ctx(const nlte_column* c);
size_t column_bytes(const nlte_column* c);
ColDev* column_dev_ptr(const nlte_column* c);
struct HostProblem;
nlte_status problem_copy(const nlte_atmos_desc* A, const nlte_atom_desc* M, const nlte_grid_desc* G,
                         const double* C_up, int32_t precision, HostProblem** out);
size_t problem_bytes(const HostProblem* H);
nlte_status problem_create_column(nlte_ctx* ctx, const HostProblem* H, hipStream_t s,
                                  void* pool_arena, size_t pool_cap, nlte_column** out);
void problem_free(HostProblem* H);
}  // namespace nlte

using namespace nlte;

namespace {

constexpr int kSteps = 4;  // device steps between state read-backs

enum ReqState { kQueued = 0, kActive = 1, kDone = 2 };

struct Request {
  uint64_t ticket = 0;
  nlte_column* col = nullptr;
  const double* n0 = nullptr;
  size_t bytes = 0;
  int state = kQueued;
  nlte_server_result res{};
  HostProblem* prob = nullptr;  // problem requests: the description, until destruction
  double* n_out = nullptr;      // problem requests: where the populations go at retirement
  void* arena = nullptr;        // problem requests: the pooled arena lent to the column
  size_t arena_cap = 0;
  ~Request() {
    if (prob) problem_free(prob);
  }
};

// Device buffer that only grows.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  hipError_t fit(size_t n) {
    if (n <= cap) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return e;
      p = nullptr;
    }
    size_t c = cap ? cap : 64;
    while (c < n) c *= 2;
    hipError_t e = hipMalloc(&p, c * sizeof(T));
    if (e == hipSuccess) cap = c;
    return e;
  }
  ~DevBuf() {
    if (p) hipFree(p);
  }
};

double now_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct nlte_server {
  nlte_ctx* ctx = nullptr;
  int device = 0;  // ctx->device, kept so that the worker and destruction never read ctx
  size_t budget = 0;
  int max_active = 0;
  nlte_solve_opts opts{};
  hipStream_t stream = nullptr;
  hipStream_t copy_stream = nullptr;
  hipStream_t setup_stream = nullptr;  // column setup of admitted requests, beside the steps
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv;       // work arrived / stop
  std::condition_variable cv_idle;  // a request finished
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  nlte_status fail = NLTE_OK;
  nlte_server_info info{};

  // server-thread state
  std::vector<Request*> active;
  DevBuf<ColDev> d_cols;
  DevBuf<Tile> d_tiles;
  DevBuf<int4> d_rate;
  DevBuf<int2> d_pb;
  DevBuf<ColState> d_states;
  DevBuf<const double*> d_n0;
  DevBuf<int> d_done;
  DevBuf<int> d_gidx;            // per-step mode lists of the formal-solution launches
  DevBuf<Tile> d_mlist;
  DevBuf<int> d_mcount;
  ColState* h_states = nullptr;  // pinned
  size_t h_states_cap = 0;
  // Column arenas of problem requests: a retired column's arena returns to
  // this pool and the next column that fits it (within 1/16 of its need)
  // reuses it, so the serving loop does not call hipMalloc and hipFree (the
  // latter waits for the device) per request.  The arenas lent to columns in
  // flight plus the pooled ones stay within the budget: pooled arenas are
  // freed, largest first, before a new one would pass it.
  std::multimap<size_t, void*> pool;
  size_t pool_bytes = 0, lent_bytes = 0;
  BatchWork bw;
  std::thread th;

  hipError_t rebuild();
  hipError_t admit(std::vector<Request*>& adm);
  void run();
  nlte_status create_pooled(Request* r, nlte_column** out);
  void return_arena(Request* r);
  void release_pool();
};

// The column of problem request r in an arena from the pool, or in a new one.
nlte_status nlte_server::create_pooled(Request* r, nlte_column** out) {
  const size_t need = pooled_arena_bytes(r->bytes);
  void* a = nullptr;
  size_t cap = 0;
  auto it = pool.lower_bound(need);
  if (it != pool.end() && it->first <= need + need / 16) {
    cap = it->first;
    a = it->second;
    pool_bytes -= cap;
    pool.erase(it);
  } else {
    while (!pool.empty() && lent_bytes + pool_bytes + need > budget) {
      auto big = std::prev(pool.end());
      (void)hipFree(big->second);
      pool_bytes -= big->first;
      pool.erase(big);
    }
    const hipError_t he = hipMalloc(&a, need);
    if (he != hipSuccess) return set_err(NLTE_E_NOMEM, "hipMalloc(%zu) failed: %s", need, hipGetErrorString(he));
    cap = need;
  }
  // set up on its own stream (the column's creation waits for it), so that a
  // block of steps may run meanwhile
  const nlte_status cs = problem_create_column(ctx, r->prob, setup_stream, a, cap, out);
  if (cs != NLTE_OK) {
    pool.emplace(cap, a);
    pool_bytes += cap;
    return cs;
  }
  r->arena = a;
  r->arena_cap = cap;
  lent_bytes += cap;
  return NLTE_OK;
}

// After the column of r has been destroyed (nothing on the device reads it).
void nlte_server::return_arena(Request* r) {
  if (!r->arena) return;
  pool.emplace(r->arena_cap, r->arena);
  pool_bytes += r->arena_cap;
  lent_bytes -= r->arena_cap;
  r->arena = nullptr;
  r->arena_cap = 0;
}

void nlte_server::release_pool() {
  for (auto& kv : pool) (void)hipFree(kv.second);
  pool.clear();
  pool_bytes = 0;
}

hipError_t nlte_server::rebuild() {
  const int n = (int)active.size();
  bw = BatchWork{};
  if (n == 0) return hipSuccess;
  std::vector<ColDev> hc(n);
  for (int c = 0; c < n; ++c) hc[c] = column_dev(active[c]->col);
  std::vector<Tile> tiles;
  std::vector<TileGroup> groups;
  std::vector<int4> rate;
  std::vector<int2> pb;
  int maxL = 0;
  const int nrate0 = build_work_lists(hc.data(), n, tiles, groups, rate, pb, maxL);
  hipError_t e;
  if ((e = d_cols.fit(n)) != hipSuccess) return e;
  if ((e = d_tiles.fit(std::max<size_t>(1, tiles.size()))) != hipSuccess) return e;
  if ((e = d_rate.fit(std::max<size_t>(1, rate.size()))) != hipSuccess) return e;
  if ((e = d_pb.fit(std::max<size_t>(1, pb.size()))) != hipSuccess) return e;
  if ((e = d_states.fit(n)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_cols.p, hc.data(), n * sizeof(ColDev), hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_tiles.p, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_rate.p, rate.data(), rate.size() * sizeof(int4), hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_pb.p, pb.data(), pb.size() * sizeof(int2), hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
  if ((size_t)n > h_states_cap) {
    if (h_states) hipHostFree(h_states);
    h_states = nullptr;
    h_states_cap = 0;
    size_t c = 64;
    while (c < (size_t)n) c *= 2;
    if ((e = hipHostMalloc((void**)&h_states, c * sizeof(ColState), hipHostMallocDefault)) != hipSuccess) return e;
    h_states_cap = c;
  }
  bw.cols = d_cols.p;
  bw.tiles = d_tiles.p;
  bw.rate_work = d_rate.p;
  bw.pb_work = d_pb.p;
  bw.ncol = n;
  bw.ntiles = (int)tiles.size();
  bw.nrate = (int)rate.size();
  bw.nrate0 = nrate0;
  bw.npb = (int)pb.size();
  bw.any_newton = 1;
  bw.any_tangent = opts.jv_method == NLTE_JV_TANGENT;
  if (!set_groups(bw, groups)) return hipErrorInvalidValue;
  for (int c = 0; c < n; ++c) {
    bw.maxnz = std::max(bw.maxnz, hc[c].nz);
    if (hc[c].prec == NLTE_FP64) bw.any64 = 1; else bw.any32 = 1;
  }
  bw.fallback = opts.fp64_fallback > 0 && bw.any32;
  std::vector<int> gidx;
  set_mode_groups(bw, tiles, n, gidx);
  if ((e = d_gidx.fit(n)) != hipSuccess) return e;
  if ((e = d_mlist.fit(4 * std::max<size_t>(1, tiles.size()))) != hipSuccess) return e;
  if ((e = d_mcount.fit(4 * kMaxGroups)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_gidx.p, gidx.data(), n * sizeof(int), hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
  bw.gidx = d_gidx.p;
  bw.mlist = d_mlist.p;
  bw.mcount = d_mcount.p;
  return hipSuccess;
}

// Newly admitted requests sit at the end of `active`; the work lists are
// already rebuilt.  Initialise their solver state (n0 or LTE).
hipError_t nlte_server::admit(std::vector<Request*>& adm) {
  const int na = (int)adm.size();
  if (!na) return hipSuccess;
  std::vector<const double*> n0(na);
  for (int i = 0; i < na; ++i) n0[i] = adm[i]->n0;
  hipError_t e;
  if ((e = d_n0.fit(na)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_n0.p, n0.data(), na * sizeof(const double*), hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
  const int first = (int)active.size() - na;
  e = solver_init(d_cols.p + first, na, d_n0.p, nullptr, opts, stream);
  if (e != hipSuccess || opts.init != 2) return e;
  // radiation-free start (Sect. 2.2.1): per admitted column, over its LTE
  // initial populations
  for (int i = 0; i < na; ++i) {
    if (adm[i]->n0) continue;  // a request that brings n0 starts from it
    zero_radiation_into(column_dev_ptr(adm[i]->col), column_dev(adm[i]->col), stream);
  }
  return hipGetLastError();
}

void nlte_server::run() {
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = d_done.fit(1);
  if (e == hipSuccess) e = hipMemsetAsync(d_done.p, 0, sizeof(int), stream);
  bool dirty = false;
  // Requests admitted while the previous block of steps ran: their columns
  // are made (on setup_stream) and they join the lists before the next block.
  std::vector<Request*> pending;
  while (e == hipSuccess) {
    if (!pending.empty() || dirty) {
      active.insert(active.end(), pending.begin(), pending.end());
      if ((e = rebuild()) != hipSuccess) break;
      if ((e = admit(pending)) != hipSuccess) break;
      pending.clear();
      dirty = false;
    }
    // the next block of steps; the host admits and sets up new requests
    // while it runs
    const int n = (int)active.size();
    const double tb = now_ms(t0);
    for (int r = 0; r < kSteps && n > 0 && e == hipSuccess; ++r) {
      e = launch_residual(bw, stream);
      if (e == hipSuccess) e = solver_step(bw.cols, nullptr, n, d_done.p, stream);
    }
    if (n > 0 && e == hipSuccess) e = solver_gather(bw.cols, n, d_states.p, stream);
    if (n > 0 && e == hipSuccess)
      e = hipMemcpyAsync(h_states, d_states.p, n * sizeof(ColState), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) break;
    std::vector<Request*> adm;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (n == 0 && queue.empty()) {
        cv_idle.notify_all();
        cv.wait(lk, [&] { return stop || !queue.empty(); });
      }
      if (stop) break;
      size_t bytes = (size_t)info.active_bytes;
      while (!queue.empty() && (int)(active.size() + pending.size() + adm.size()) < max_active) {
        Request* r = queue.front();
        const bool empty = active.empty() && pending.empty() && adm.empty();
        if (!empty && bytes + r->bytes > budget) break;
        queue.pop_front();
        r->state = kActive;
        r->res.t_admit_ms = now_ms(t0);
        bytes += r->bytes;
        adm.push_back(r);
      }
      info.active_bytes = (int64_t)bytes;
      info.peak_active_bytes = std::max(info.peak_active_bytes, info.active_bytes);
      info.queued = (int32_t)queue.size();
    }
    // problem requests: their columns are made now, within the budget
    for (Request* r : adm) {
      if (r->prob && !r->col) {
        nlte_column* c = nullptr;
        const nlte_status cs = create_pooled(r, &c);
        if (cs != NLTE_OK) {
          std::lock_guard<std::mutex> lk(mu);
          r->res.stats = nlte_solve_stats{};
          r->res.stats.status = cs;
          r->res.t_done_ms = now_ms(t0);
          r->state = kDone;
          info.active_bytes -= (int64_t)r->bytes;
          info.completed += 1;
          cv_idle.notify_all();
          continue;
        }
        r->col = c;
      }
      pending.push_back(r);
    }
    if (n == 0) continue;
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) break;
    // problem requests that finished: populations to the caller's buffer,
    // then the column goes and its arena returns to the pool
    bool freed = false;
    for (int c = 0; c < n && e == hipSuccess; ++c) {
      Request* r = active[c];
      if (r->prob && state_done(h_states[c])) {
        const ColDev& C = column_dev(r->col);
        if (r->n_out)
          e = hipMemcpyAsync(r->n_out, C.n, (size_t)C.N * sizeof(double), hipMemcpyDeviceToDevice, stream);
        freed = true;
      }
    }
    if (freed && e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) break;
    for (int c = 0; c < n; ++c) {
      Request* r = active[c];
      if (r->prob && r->col && state_done(h_states[c])) {
        nlte_column_destroy(r->col);
        r->col = nullptr;
        return_arena(r);
      }
    }
    const double t = now_ms(t0);
    std::vector<Request*> still;
    still.reserve(n);
    {
      std::lock_guard<std::mutex> lk(mu);
      info.steps += kSteps;
      info.busy_ms += t - tb;
      for (int c = 0; c < n; ++c) {
        Request* r = active[c];
        if (state_done(h_states[c])) {
          state_stats(h_states[c], &r->res.stats);
          r->res.t_done_ms = t;
          r->state = kDone;
          info.active_bytes -= (int64_t)r->bytes;
          info.completed += 1;
          dirty = true;
        } else {
          still.push_back(r);
        }
      }
      info.active = (int32_t)still.size();
    }
    if (dirty) cv_idle.notify_all();
    active.swap(still);
  }
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    fail = NLTE_E_DEVICE;
    for (auto& kv : reqs) {
      Request* r = kv.second;
      if (r->state != kDone) {
        r->state = kDone;
        r->res.stats.status = NLTE_E_DEVICE;
        r->res.t_done_ms = now_ms(t0);
      }
    }
    queue.clear();
    active.clear();
    cv_idle.notify_all();
  }
}

extern "C" nlte_status nlte_server_create(nlte_ctx* ctx, size_t hbm_budget, int32_t max_active,
                                          const nlte_solve_opts* opts, nlte_server** out) {
  if (!ctx || !out || hbm_budget == 0 || max_active < 1)
    return set_err(NLTE_E_INVALID, "bad server arguments");
  nlte_solve_opts o;
  nlte_solve_opts_default(&o);
  if (opts) o = *opts;
  const nlte_status vs = check_solve_opts(o);
  if (vs != NLTE_OK) return vs;
  if (o.init == 0)
    return set_err(NLTE_E_INVALID, "server requests start from n0 when they bring one, else from "
                                   "LTE (opts.init = 1) or the radiation-free populations (2)");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(NLTE_E_DEVICE, "hipSetDevice failed");
  nlte_server* S = new nlte_server();
  S->ctx = ctx;
  S->device = ctx->device;
  S->budget = hbm_budget;
  S->max_active = max_active;
  S->opts = o;
  S->t0 = std::chrono::steady_clock::now();
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->setup_stream, hipStreamNonBlocking) != hipSuccess) {
    if (S->stream) hipStreamDestroy(S->stream);
    if (S->copy_stream) hipStreamDestroy(S->copy_stream);
    delete S;
    return set_err(NLTE_E_DEVICE, "stream creation failed");
  }
  S->th = std::thread([S] { S->run(); });
  *out = S;
  return NLTE_OK;
}

extern "C" nlte_status nlte_server_submit(nlte_server* S, nlte_column* col, const double* n0_dev,
                                          uint64_t* ticket) {
  if (!S || !col || !ticket) return set_err(NLTE_E_INVALID, "NULL argument");
  if (column_ctx(col) != S->ctx) return set_err(NLTE_E_INVALID, "column from another context");
  Request* r = new Request();
  r->col = col;
  r->n0 = n0_dev;
  r->bytes = column_bytes(col);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fail != NLTE_OK) {
      delete r;
      return set_err(S->fail, "server stopped after a device error");
    }
    for (auto& kv : S->reqs)
      if (kv.second->col == col) {
        delete r;
        return set_err(NLTE_E_INVALID, "column already submitted (ticket %llu)",
                       (unsigned long long)kv.first);
      }
    r->ticket = S->next_ticket++;
    r->res.t_submit_ms = now_ms(S->t0);
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
    S->info.submitted += 1;
    S->info.queued = (int32_t)S->queue.size();
  }
  S->cv.notify_one();
  *ticket = r->ticket;
  return NLTE_OK;
}

extern "C" nlte_status nlte_server_submit_problem(nlte_server* S, const nlte_atmos_desc* atmos,
                                                  const nlte_atom_desc* atom,
                                                  const nlte_grid_desc* grid, const double* C_up,
                                                  int32_t precision, double* n_out_dev,
                                                  uint64_t* ticket) {
  if (!S || !ticket || !n_out_dev) return set_err(NLTE_E_INVALID, "NULL argument");
  HostProblem* H = nullptr;
  const nlte_status ps = problem_copy(atmos, atom, grid, C_up, precision, &H);
  if (ps != NLTE_OK) return ps;
  Request* r = new Request();
  r->prob = H;
  r->n_out = n_out_dev;
  r->bytes = problem_bytes(H);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fail != NLTE_OK) {
      delete r;
      return set_err(S->fail, "server stopped after a device error");
    }
    r->ticket = S->next_ticket++;
    r->res.t_submit_ms = now_ms(S->t0);
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
    S->info.submitted += 1;
    S->info.queued = (int32_t)S->queue.size();
  }
  S->cv.notify_one();
  *ticket = r->ticket;
  return NLTE_OK;
}

extern "C" nlte_status nlte_server_poll(nlte_server* S, uint64_t ticket, double* n_out_dev,
                                        nlte_server_result* res) {
  if (!S) return set_err(NLTE_E_INVALID, "NULL server");
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return set_err(NLTE_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state != kDone) return set_err(NLTE_E_BUSY, "ticket %llu not finished", (unsigned long long)ticket);
    r = it->second;
    S->reqs.erase(it);
  }
  nlte_status st = NLTE_OK;
  if (n_out_dev && !r->prob && r->res.stats.status != NLTE_E_DEVICE) {
    const ColDev& C = column_dev(r->col);
    if (hipMemcpyAsync(n_out_dev, C.n, (size_t)C.N * sizeof(double), hipMemcpyDeviceToDevice,
                       S->copy_stream) != hipSuccess ||
        hipStreamSynchronize(S->copy_stream) != hipSuccess)
      st = set_err(NLTE_E_DEVICE, "copy of the result failed");
  }
  if (res) *res = r->res;
  delete r;
  return st;
}

extern "C" nlte_status nlte_server_drain(nlte_server* S, double timeout_s) {
  if (!S) return set_err(NLTE_E_INVALID, "NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  const auto until = std::chrono::steady_clock::now() +
                     std::chrono::microseconds((long long)(timeout_s * 1e6));
  const bool ok = S->cv_idle.wait_until(lk, until, [&] {
    return S->fail != NLTE_OK || (S->queue.empty() && S->info.completed == S->info.submitted);
  });
  if (S->fail != NLTE_OK) return set_err(S->fail, "server stopped after a device error");
  return ok ? NLTE_OK : set_err(NLTE_E_BUSY, "drain timed out");
}

extern "C" nlte_status nlte_server_info_get(const nlte_server* S, nlte_server_info* out) {
  if (!S || !out) return set_err(NLTE_E_INVALID, "NULL argument");
  nlte_server* m = const_cast<nlte_server*>(S);
  std::lock_guard<std::mutex> lk(m->mu);
  *out = m->info;
  return NLTE_OK;
}

extern "C" void nlte_server_destroy(nlte_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  (void)hipSetDevice(S->device);
  hipStreamSynchronize(S->stream);
  for (auto& kv : S->reqs) {
    Request* r = kv.second;
    if (r->prob && r->col) nlte_column_destroy(r->col);
    if (r->arena) (void)hipFree(r->arena);
    delete r;
  }
  S->release_pool();
  if (S->h_states) hipHostFree(S->h_states);
  hipStreamDestroy(S->stream);
  hipStreamDestroy(S->copy_stream);
  hipStreamDestroy(S->setup_stream);
  delete S;
}
