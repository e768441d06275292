// Host side of the ensemble entry points (nf_batch_*, include/nf.h).
//
// Each instance owns the workspace of one nf_grid.  The instances are split
// into partitions; a partition has its own HIP stream and host thread, and
// its instances' status blocks are moved into one contiguous array so that a
// single copy polls them all.  Within a partition, instances of equal grid
// shape form a launch group: every pass of the time step (Algorithm 1) and
// every PCG iteration is one launch per group, with the instance as the second
// grid dimension and its pointers and parameters read from a device table of
// per-instance argument structs.  The kernel bodies are those of the
// single-instance entry points, so each instance computes exactly what nf_run
// computes for it, whatever the partition.
//
// The partition count is tuned: unless the caller fixes it, the first
// nf_batch_run times two steps of every candidate count on scratch copies of
// m and p and keeps the fastest.  Different partitions overlap one another's
// transform and memory phases, which identical kernels of one launch cannot.
// Optionally (nf_batch_set_graphs) a partition records each chunk of PCG
// iterations as a HIP graph and replays it in later solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "nf.h"
#include "nf_handle.h"
#include "nf_internal.h"

using namespace nf;

namespace {

thread_local std::string batch_create_err;

// device argument tables of one launch group (k entries each)
struct Tables {
  FluxArgs *flux_init = nullptr, *flux_init_lo = nullptr, *flux_loop = nullptr, *flux32 = nullptr;
  DivArgs *div64 = nullptr, *div32 = nullptr;
  UpdArgs *upd64 = nullptr, *upd32 = nullptr;
  ColGradArgs *grad_x = nullptr, *split_p = nullptr, *split_g = nullptr;
  SplitArgs* split = nullptr;
  HeatArgs* heat = nullptr;
  FinalArgs* fin = nullptr;
  RefStartArgs* rstart = nullptr;
  RefAccArgs* racc = nullptr;
  SumArgs *sum_rr = nullptr, *sum_dm = nullptr;
};

// One partition: a subset of the instances, with its own stream and statuses.
struct Part {
  int count = 0;
  int dtype = NF_F64;
  hipStream_t stream = nullptr;  // owned
  std::vector<nf_grid*> inst;    // not owned
  std::vector<int> gidx;         // ensemble index of each instance
  DevStatus* st = nullptr;   // count contiguous statuses
  DevStatus* hst = nullptr;  // pinned, 2 * count
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct Group {
    std::vector<int> idx;
    Geo shape;
    char* dev = nullptr;
    size_t bytes = 0;
    std::vector<char> host;
    Tables t;
  };
  std::vector<Group> groups;
  std::vector<DevStatus> fin;
  int last_iters = 0;
  int last_inner[4] = {0, 0, 0, 0};
  std::string err;
  // PCG iteration chunks recorded as HIP graphs, keyed by (first iteration,
  // iterations, FP32 inner solve, max_iter, tol2 bits)
  bool use_graphs = false;
  std::map<std::tuple<int, int, int, int, uint64_t>, hipGraphExec_t> graphs;
};

}  // namespace

struct nf_batch {
  int count = 0;
  int dtype = NF_F64;
  hipStream_t stream = nullptr;   // the caller's stream
  std::vector<nf_grid*> inst;     // owned
  std::vector<Part*> parts;
  int nparts = 0;                 // 0: tune at the next run
  hipEvent_t fork = nullptr;
  std::vector<double> tune_ms;    // step time of each candidate count (index = count - 1)
  bool use_graphs = false;
  std::string err;
};

namespace {

int bfail(Part* b, int code, const std::string& msg) {
  b->err = msg;
  return code;
}

#define BCHK(b, expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return bfail((b), NF_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_));    \
  } while (0)

// Offsets of the tables in a group's allocation (256-byte aligned).
struct Layout {
  size_t off[18];
  size_t total;
};
Layout layout(int k) {
  const size_t sz[18] = {sizeof(FluxArgs),    sizeof(FluxArgs),     sizeof(FluxArgs),    sizeof(FluxArgs),
                         sizeof(DivArgs),     sizeof(DivArgs),      sizeof(UpdArgs),     sizeof(UpdArgs),
                         sizeof(ColGradArgs), sizeof(ColGradArgs),  sizeof(ColGradArgs), sizeof(SplitArgs),
                         sizeof(HeatArgs),    sizeof(FinalArgs),    sizeof(RefStartArgs), sizeof(RefAccArgs),
                         sizeof(SumArgs),     sizeof(SumArgs)};
  Layout L;
  size_t o = 0;
  for (int i = 0; i < 18; ++i) {
    L.off[i] = o;
    o += (sz[i] * k + 255) & ~(size_t)255;
  }
  L.total = o;
  return L;
}

template <typename T>
T* at(char* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

void bind_tables(Part::Group& G, char* base, const Layout& L) {
  Tables& t = G.t;
  t.flux_init = at<FluxArgs>(base, L.off[0]);
  t.flux_init_lo = at<FluxArgs>(base, L.off[1]);
  t.flux_loop = at<FluxArgs>(base, L.off[2]);
  t.flux32 = at<FluxArgs>(base, L.off[3]);
  t.div64 = at<DivArgs>(base, L.off[4]);
  t.div32 = at<DivArgs>(base, L.off[5]);
  t.upd64 = at<UpdArgs>(base, L.off[6]);
  t.upd32 = at<UpdArgs>(base, L.off[7]);
  t.grad_x = at<ColGradArgs>(base, L.off[8]);
  t.split_p = at<ColGradArgs>(base, L.off[9]);
  t.split_g = at<ColGradArgs>(base, L.off[10]);
  t.split = at<SplitArgs>(base, L.off[11]);
  t.heat = at<HeatArgs>(base, L.off[12]);
  t.fin = at<FinalArgs>(base, L.off[13]);
  t.rstart = at<RefStartArgs>(base, L.off[14]);
  t.racc = at<RefAccArgs>(base, L.off[15]);
  t.sum_rr = at<SumArgs>(base, L.off[16]);
  t.sum_dm = at<SumArgs>(base, L.off[17]);
}

// Fill the host image of a group's tables for one run and copy it to the device.
int upload_tables(Part* b, Part::Group& G, const nf_params* prm, double dt, double* const* m,
                  double* const* p, const double* const* r) {
  const int k = (int)G.idx.size();
  const Layout L = layout(k);
  char* hb = G.host.data();
  Part::Group H;  // host-side view of the same layout
  bind_tables(H, hb, L);
  for (int j = 0; j < k; ++j) {
    const int i = G.idx[j];
    nf_grid* g = b->inst[i];
    const size_t n = (size_t)g->nx * g->ny;
    const Geo& g64 = g->geo;
    const Geo& g32 = g->geo32;
    H.t.flux_init[j] = FluxArgs{g64, g->mix[0], g->mix[1], m[i], r[i], slot_ptr(g->part, SLOT_KBAR), nullptr};
    H.t.flux_init_lo[j] = FluxArgs{g64, g->mix[0], g->mix[1], m[i], r[i], slot_ptr(g->part, SLOT_KBAR), g->lo};
    H.t.flux_loop[j] = FluxArgs{g64, g->mix[0], g->mix[1], m[i], r[i], nullptr, nullptr};
    H.t.flux32[j] = FluxArgs{g32, g->mix32[0], g->mix32[1], g->lo, g->lo ? g->lo + 2 * n : nullptr, nullptr, nullptr};
    H.t.div64[j] = DivArgs{g64, g->mix[0], g->mix[1], g->qh, g->dh, g->rh, g->bh};
    H.t.div32[j] = DivArgs{g32, g->mix32[0], g->mix32[1], g->q32, g->d32, g->r32, nullptr};
    H.t.upd64[j] = UpdArgs{g64, g->xh, g->rh, g->dh, g->qh, g->mix[0], g->mix[1]};
    H.t.upd32[j] = UpdArgs{g32, g->x32, g->r32, g->d32, g->q32, g->mix32[0], g->mix32[1]};
    H.t.grad_x[j] = ColGradArgs{g64, g->xh, nullptr, g->mix[0], g->mix[1]};
    H.t.split_p[j] = ColGradArgs{g64, g->xh, g->mix[0], nullptr, nullptr};
    H.t.split_g[j] = ColGradArgs{g64, g->xh, nullptr, g->mix[1], g->mix[2]};
    H.t.split[j] = SplitArgs{g64,        g->mix[0], g->mix[1],        g->mix[2],       m[i],
                             p[i],       prm[i].c2 * dt, prm[i].gamma, dt, std::exp(-dt)};
    H.t.heat[j] = HeatArgs{g64, g->mix[0], g->mix[1], prm[i].D2 * dt, nullptr};
    H.t.fin[j] = FinalArgs{g64, g->mix[0], g->mix[1], m[i], slot_ptr(g->part, SLOT_DM)};
    H.t.rstart[j] = RefStartArgs{g32, g->rh, g->xh, g->x32, g->r32, g->d32, g->mix32[0], g->mix32[1]};
    H.t.racc[j] = RefAccArgs{g64, g->xh, g->x32, g->mix[0], g->mix[1]};
    H.t.sum_rr[j] = SumArgs{slot_ptr(g->part, SLOT_RR), g->st};
    H.t.sum_dm[j] = SumArgs{slot_ptr(g->part, SLOT_DM), g->st};
  }
  BCHK(b, hipMemcpyAsync(G.dev, hb, L.total, hipMemcpyHostToDevice, b->stream));
  return NF_OK;
}

int read_all(Part* b) {
  BCHK(b, hipMemcpyAsync(b->fin.data(), b->st, sizeof(DevStatus) * b->count, hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  return NF_OK;
}

// Iterations it0 .. it0 + nk - 1 of the PCG loop of every launch group (kernel
// launches only, so that the sequence can be recorded as a graph).
int launch_chunk(Part* b, bool f32, int it0, int nk, int max_iter, double tol2) {
  hipStream_t s = b->stream;
  for (int it = it0; it < it0 + nk; ++it) {
    for (auto& G : b->groups) {
      const int k = (int)G.idx.size();
      BCHK(b, launchb_row_flux(G.shape, f32, f32 ? G.t.flux32 : G.t.flux_loop, k, it, tol2, s));
      BCHK(b, launchb_col_div(G.shape, f32, false, f32 ? G.t.div32 : G.t.div64, k, it, s));
      BCHK(b, launchb_col_update(G.shape, f32, f32 ? G.t.upd32 : G.t.upd64, k, 0, it + 1, max_iter, tol2, s));
    }
  }
  return NF_OK;
}

void graphs_clear(Part* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// A chunk of iterations, replayed from its recorded graph (recorded on first
// use).  The launches read their per-instance arguments from the group tables,
// whose device addresses are fixed for the partition and whose contents each
// run uploads before the first chunk, so a recording stays valid across runs.
int run_chunk(Part* b, bool f32, int it0, int nk, int max_iter, double tol2) {
  if (!b->use_graphs) return launch_chunk(b, f32, it0, nk, max_iter, tol2);
  hipStream_t s = b->stream;
  uint64_t tb;
  std::memcpy(&tb, &tol2, sizeof tb);
  const auto key = std::make_tuple(it0, nk, f32 ? 1 : 0, max_iter, tb);
  auto found = b->graphs.find(key);
  hipGraphExec_t ex = nullptr;
  if (found != b->graphs.end()) {
    ex = found->second;
  } else {
    if (b->graphs.size() >= 256) graphs_clear(b);
    BCHK(b, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int rc = launch_chunk(b, f32, it0, nk, max_iter, tol2);
    hipGraph_t gr = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &gr);
    if (rc != NF_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    BCHK(b, ee);
    const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    BCHK(b, ie);
    b->graphs[key] = ex;
  }
  BCHK(b, hipGraphLaunch(ex, s));
  return NF_OK;
}

// PCG iterations of all instances, chunked and polled as in the single-instance
// loop; stops once every instance's status reports a stop.  The polled copy
// that shows every stop is final (no later launch of the loop writes a stopped
// instance's status), so b->fin is taken from it without waiting for the
// queued no-op tail; later launches queue behind that tail.
int batch_loop(Part* b, bool f32, int max_iter, double tol2, int expect) {
  hipStream_t s = b->stream;
  const int c = b->count;
  int it = 0, slot = 0, pending = -1;
  bool first_chunk = true;
  while (it < max_iter) {
    // up to one iteration short of the last solve's count, then one iteration per
    // chunk: the host polls one chunk behind, so at most about one chunk of
    // launches is queued past the stop (they return at once)
    int nk = first_chunk ? (expect > 3 ? expect - 1 : 2) : 1;
    first_chunk = false;
    if (nk > max_iter - it) nk = max_iter - it;
    const int rc = run_chunk(b, f32, it, nk, max_iter, tol2);
    if (rc != NF_OK) return rc;
    it += nk;
    BCHK(b, hipMemcpyAsync(b->hst + (size_t)slot * c, b->st, sizeof(DevStatus) * c, hipMemcpyDeviceToHost, s));
    BCHK(b, hipEventRecord(b->ev[slot], s));
    if (pending >= 0) {
      BCHK(b, poll_event(b->ev[pending]));
      bool all = true;
      for (int i = 0; i < c && all; ++i) all = b->hst[(size_t)pending * c + i].conv_at != INT_MAX;
      if (all) {
        std::memcpy(b->fin.data(), b->hst + (size_t)pending * c, sizeof(DevStatus) * c);
        return NF_OK;
      }
    }
    pending = slot;
    slot ^= 1;
  }
  return read_all(b);
}

struct SolveRes {
  std::vector<int> iters, converged;
};

// Pressure solves of all instances (the pcg / pcg_refined sequence of the
// single-instance path, batched).  first: warm start from p, else from the
// spectral iterate kept from the previous solve.
int batch_solve(Part* b, bool first, double* const* p, double rtol, int max_iter, SolveRes* out) {
  hipStream_t s = b->stream;
  const int c = b->count;
  BCHK(b, launchb_status_reset(b->st, c, 0, s));
  if (first) {
    for (int i = 0; i < c; ++i) {
      nf_grid* g = b->inst[i];
      BCHK(b, launch_row_r2c(g->geo, p[i], g->mix[0], nullptr, s));
      BCHK(b, launch_col_fwd(g->geo, g->mix[0], g->xh, 1, g->mix[0], g->mix[1], s));
    }
  } else {
    for (auto& G : b->groups) BCHK(b, launchb_col_grad(G.shape, G.t.grad_x, (int)G.idx.size(), true, s));
  }
  const double tol2 = rtol * rtol;
  out->iters.assign(c, 0);
  out->converged.assign(c, 0);
  if (b->dtype == NF_F64) {
    for (auto& G : b->groups) {
      const int k = (int)G.idx.size();
      BCHK(b, launchb_row_flux(G.shape, false, G.t.flux_init, k, -1, 0.0, s));
      BCHK(b, launchb_col_div(G.shape, false, true, G.t.div64, k, 0, s));
      BCHK(b, launchb_col_update(G.shape, false, G.t.upd64, k, 1, 0, max_iter, tol2, s));
    }
    int rc = batch_loop(b, false, max_iter, tol2, b->last_iters);
    if (rc) return rc;
    // final convergence test of solves stopped by max_iter, on the last residual
    bool capped = false;
    for (int i = 0; i < c; ++i) {
      const DevStatus& f = b->fin[i];
      capped = capped || (!f.converged && f.conv_at == max_iter && max_iter > 0 &&
                          !(f.flags & (FLAG_NONFINITE | FLAG_INCOMPAT)));
    }
    if (capped) {
      for (auto& G : b->groups)
        BCHK(b, launchb_sum_slot(G.t.sum_rr, (int)G.idx.size(), 1, rr_nwg(G.shape, false), 11, s));
      rc = read_all(b);
      if (rc) return rc;
    }
    int mx = 0;
    for (int i = 0; i < c; ++i) {
      const DevStatus& f = b->fin[i];
      bool conv = f.converged != 0;
      if (!conv && f.conv_at == max_iter && max_iter > 0 && !(f.flags & (FLAG_NONFINITE | FLAG_INCOMPAT)))
        conv = f.out[11] <= tol2 * f.bb;
      out->iters[i] = f.iters;
      out->converged[i] = conv ? 1 : 0;
      mx = f.iters > mx ? f.iters : mx;
    }
    if (mx > 0) b->last_iters = mx;
    return NF_OK;
  }
  for (int outer = 0;; ++outer) {
    for (auto& G : b->groups) {
      const int k = (int)G.idx.size();
      BCHK(b, launchb_row_flux(G.shape, false, outer == 0 ? G.t.flux_init_lo : G.t.flux_init, k, -1, 0.0, s));
      BCHK(b, launchb_col_div(G.shape, false, true, G.t.div64, k, 0, s));
      BCHK(b, launchb_col_refine_start(G.shape, G.t.rstart, k, tol2, b->inst[G.idx[0]]->inner_floor, max_iter, s));
    }
    const int slot = outer < 3 ? outer : 3;
    int rc = batch_loop(b, true, max_iter, 1.0, b->last_inner[slot]);
    if (rc) return rc;
    bool all = true;
    int mx = 0;
    for (int i = 0; i < c; ++i) {
      all = all && b->fin[i].outer_done;
      mx = b->fin[i].iters > mx ? b->fin[i].iters : mx;
    }
    if (all) break;
    if (mx > 0) b->last_inner[slot] = mx;
    for (auto& G : b->groups) BCHK(b, launchb_col_refine_acc(G.shape, G.t.racc, (int)G.idx.size(), s));
  }
  for (int i = 0; i < c; ++i) {
    out->iters[i] = b->fin[i].itot;
    out->converged[i] = b->fin[i].converged;
  }
  return NF_OK;
}

}  // namespace

namespace {

// Host-side meeting point of the partitions after the first solve and after
// every step: a stop reported by any partition (incompatible S, non-finite
// activation, a device error) stops all of them at the same point, as in a
// single-partition run.  A partition that returns early leaves the barrier.
struct StepSync {
  std::mutex mu;
  std::condition_variable cv;
  int live;
  int arrived = 0;
  int64_t gen = 0;
  bool flag = false, last = false, sticky = false;
  explicit StepSync(int k) : live(k) {}
  void complete() {
    last = flag || sticky;
    flag = false;
    arrived = 0;
    ++gen;
    cv.notify_all();
  }
  // report this partition's stop condition; true if any partition stops
  bool arrive(bool stop) {
    std::unique_lock<std::mutex> lk(mu);
    flag = flag || stop;
    const int64_t g = gen;
    if (++arrived >= live) {
      complete();
      return last;
    }
    cv.wait(lk, [&] { return gen != g; });
    return last;
  }
  void leave(bool error) {
    std::lock_guard<std::mutex> lk(mu);
    sticky = sticky || error;
    --live;
    if (arrived > 0 && arrived >= live) complete();
  }
};

// returned by a partition that stopped because another one did
constexpr int NF_STOPPED_BY_OTHER = 1;

// nf_batch_run for the instances of one partition (arrays indexed locally).
int part_run(Part* b, StepSync* sync, const nf_params* prm, double dt, int64_t steps, double* const* m,
             double* const* p, const double* const* r, const double* const* S, double rtol, int max_iter,
             nf_run_info* info) {
  b->err.clear();
  const int c = b->count;
  hipStream_t s = b->stream;
  std::vector<nf_run_info> ri(c);
  for (auto& x : ri) {
    x.steps = 0;
    x.stop_reason = NF_STOP_MAX_STEPS;
    x.last_dm = NAN;
    x.last_energy = NAN;
    x.prev_energy = NAN;
    x.total_cg_iters = 0;
    x.unconverged_solves = 0;
  }
  auto finish = [&](int rc) {
    if (info)
      for (int i = 0; i < c; ++i) info[i] = ri[i];
    return rc;
  };
  for (auto& G : b->groups) {
    const int rc = upload_tables(b, G, prm, dt, m, p, r);
    if (rc) return finish(rc);
  }
  BCHK(b, launchb_status_reset(b->st, c, 1, s));
  for (int i = 0; i < c; ++i) {
    nf_grid* g = b->inst[i];
    BCHK(b, launch_row_r2c(g->geo, S[i], g->mix[0], slot_ptr(g->part, SLOT_SCHK), s));
    BCHK(b, launch_col_fwd(g->geo, g->mix[0], g->bh, 0, nullptr, nullptr, s));
  }
  SolveRes sr;
  int rc = batch_solve(b, true, p, rtol, max_iter, &sr);
  if (rc) return finish(rc);
  for (int i = 0; i < c; ++i) {
    ri[i].total_cg_iters += sr.iters[i];
    if (b->fin[i].flags & FLAG_INCOMPAT) {
      ri[i].stop_reason = NF_STOP_ERROR;
      rc = bfail(b, NF_EINCOMPAT, "instance " + std::to_string(b->gidx[i]) + ": S violates the solvability condition");
    } else if (!sr.converged[i]) {
      ri[i].unconverged_solves++;
    }
  }
  if (sync->arrive(rc != NF_OK) && rc == NF_OK) return finish(NF_STOPPED_BY_OTHER);
  if (rc) return finish(rc);
  for (int64_t step = 0; step < steps; ++step) {
    for (auto& G : b->groups) {
      const int k = (int)G.idx.size();
      BCHK(b, launchb_col_grad(G.shape, G.t.split_p, k, false, s));
      BCHK(b, launchb_col_grad(G.shape, G.t.split_g, k, true, s));
      BCHK(b, launchb_row_split(G.shape, G.t.split, k, s));
      BCHK(b, launchb_col_heat(G.shape, G.t.heat, k, s));
      BCHK(b, launchb_row_final(G.shape, G.t.fin, k, s));
    }
    rc = batch_solve(b, false, p, rtol, max_iter, &sr);
    if (rc) return finish(rc);
    bool bad = false;
    for (int i = 0; i < c; ++i) {
      ri[i].steps += 1;
      ri[i].total_cg_iters += sr.iters[i];
      if ((b->fin[i].flags | b->fin[i].sticky) & FLAG_NONFINITE) {
        ri[i].stop_reason = NF_STOP_ERROR;
        bad = true;
      } else if (!sr.converged[i]) {
        ri[i].unconverged_solves++;
      }
    }
    if (sync->arrive(bad) && !bad) return finish(NF_STOPPED_BY_OTHER);
    if (bad) return finish(bfail(b, NF_ENONFINITE, "activation overflow: c^2 |grad p|^2 dt too large for the time step"));
  }
  // Delta m of the last step and p = p[m_final]
  for (auto& G : b->groups)
    BCHK(b, launchb_sum_slot(G.t.sum_dm, (int)G.idx.size(), 2, row_nwg(G.shape), 8, s));
  for (int i = 0; i < c; ++i) {
    nf_grid* g = b->inst[i];
    BCHK(b, launch_col_grad(g->geo, g->xh, g->mix[0], nullptr, nullptr, s));
    BCHK(b, launch_row_c2r(g->geo, g->mix[0], p[i], s));
  }
  rc = read_all(b);
  if (rc) return finish(rc);
  for (int i = 0; i < c; ++i) {
    const DevStatus& f = b->fin[i];
    ri[i].last_dm = f.out[9] > 0.0 ? std::sqrt(f.out[8] / f.out[9]) / dt : 0.0;
    if (f.sticky & FLAG_NONFINITE) {
      ri[i].stop_reason = NF_STOP_ERROR;
      rc = bfail(b, NF_ENONFINITE, "activation overflow: c^2 |grad p|^2 dt too large for the time step");
    }
  }
  return finish(rc);
}

void part_destroy(Part* q) {
  if (!q) return;
  if (q->stream) (void)hipStreamSynchronize(q->stream);
  graphs_clear(q);
  for (auto& G : q->groups)
    if (G.dev) (void)hipFree(G.dev);
  if (q->st) (void)hipFree(q->st);
  if (q->hst) (void)hipHostFree(q->hst);
  for (int i = 0; i < 2; ++i)
    if (q->ev[i]) (void)hipEventDestroy(q->ev[i]);
  if (q->stream) (void)hipStreamDestroy(q->stream);
  delete q;
}

// A partition over the instances idx of the ensemble: its stream (default
// priority), contiguous statuses (the instances' handles point into them) and
// the launch groups of its grid shapes.
int part_create(nf_batch* top, const std::vector<int>& idx, Part** out, std::string& what) {
  *out = nullptr;
  Part* q = new Part();
  q->count = (int)idx.size();
  q->dtype = top->dtype;
  q->use_graphs = top->use_graphs;
  q->gidx = idx;
  hipError_t e = hipSuccess;
  auto fail = [&](int code, const char* call) {
    what = std::string(call) + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : "");
    part_destroy(q);
    return code;
  };
  if ((e = hipStreamCreateWithFlags(&q->stream, hipStreamNonBlocking)) != hipSuccess)
    return fail(NF_EDEVICE, "hipStreamCreateWithFlags");
  if ((e = hipMalloc((void**)&q->st, sizeof(DevStatus) * q->count)) != hipSuccess) return fail(NF_ENOMEM, "hipMalloc(st)");
  if ((e = hipMemset(q->st, 0, sizeof(DevStatus) * q->count)) != hipSuccess) return fail(NF_EDEVICE, "hipMemset(st)");
  if ((e = hipHostMalloc((void**)&q->hst, 2 * sizeof(DevStatus) * q->count, hipHostMallocDefault)) != hipSuccess)
    return fail(NF_ENOMEM, "hipHostMalloc(status)");
  for (int i = 0; i < 2; ++i)
    if ((e = hipEventCreateWithFlags(&q->ev[i], hipEventDisableTiming)) != hipSuccess)
      return fail(NF_EDEVICE, "hipEventCreate");
  q->fin.resize(q->count);
  for (int i = 0; i < q->count; ++i) {
    nf_grid* g = top->inst[idx[i]];
    q->inst.push_back(g);
    g->st = q->st + i;
    g->geo.st = g->st;
    g->geo32.st = g->st;
    Part::Group* grp = nullptr;
    for (auto& G : q->groups) {
      const nf_grid* h = q->inst[G.idx[0]];
      if (h->nx == g->nx && h->ny == g->ny && h->lx == g->lx && h->ly == g->ly) grp = &G;
    }
    if (!grp) {
      q->groups.emplace_back();
      grp = &q->groups.back();
      grp->shape = g->geo;
    }
    grp->idx.push_back(i);
  }
  for (auto& G : q->groups) {
    const Layout Lo = layout((int)G.idx.size());
    G.bytes = Lo.total;
    G.host.assign(Lo.total, 0);
    if ((e = hipMalloc((void**)&G.dev, Lo.total)) != hipSuccess) return fail(NF_ENOMEM, "hipMalloc(tables)");
    bind_tables(G, G.dev, Lo);
  }
  *out = q;
  return NF_OK;
}

void parts_clear(nf_batch* b) {
  for (Part* q : b->parts) part_destroy(q);
  b->parts.clear();
  for (nf_grid* g : b->inst) {
    if (!g) continue;  // creation failed before this instance
    g->st = g->st_own;
    g->geo.st = g->st_own;
    g->geo32.st = g->st_own;
  }
}

// Split the instances into k partitions of about equal grid-point counts
// (largest instances first, each to the lightest partition; ties to the lower
// partition index, so the split is deterministic).
int parts_build(nf_batch* b, int k) {
  parts_clear(b);
  std::vector<int> order(b->count);
  for (int i = 0; i < b->count; ++i) order[i] = i;
  auto pts = [&](int i) { return (int64_t)b->inst[i]->nx * b->inst[i]->ny; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return pts(a) > pts(c); });
  std::vector<std::vector<int>> idx(k);
  std::vector<int64_t> load(k, 0);
  for (int i : order) {
    int best = 0;
    for (int j = 1; j < k; ++j)
      if (load[j] < load[best]) best = j;
    idx[best].push_back(i);
    load[best] += pts(i);
  }
  for (auto& v : idx) std::sort(v.begin(), v.end());
  for (int j = 0; j < k; ++j) {
    Part* q = nullptr;
    std::string what;
    const int rc = part_create(b, idx[j], &q, what);
    if (rc != NF_OK) {
      parts_clear(b);
      b->nparts = 0;
      b->err = "partition setup: " + what;
      return rc;
    }
    b->parts.push_back(q);
  }
  b->nparts = k;
  return NF_OK;
}

// Run every partition on its own host thread (the first on the calling one),
// after the caller's stream has reached this point.
int parts_run(nf_batch* b, const nf_params* prm, double dt, int64_t steps, double* const* m, double* const* p,
              const double* const* r, const double* const* S, double rtol, int max_iter, nf_run_info* info) {
  const int k = (int)b->parts.size();
  hipError_t e = hipEventRecord(b->fork, b->stream);
  for (int j = 0; j < k && e == hipSuccess; ++j) e = hipStreamWaitEvent(b->parts[j]->stream, b->fork, 0);
  if (e != hipSuccess) {
    b->err = std::string("fork of the partition streams: ") + hipGetErrorString(e);
    return NF_EDEVICE;
  }
  struct Args {
    std::vector<nf_params> prm;
    std::vector<double*> m, p;
    std::vector<const double*> r, S;
    std::vector<nf_run_info> info;
    int rc = NF_OK;
  };
  std::vector<Args> a(k);
  for (int j = 0; j < k; ++j) {
    for (int i : b->parts[j]->gidx) {
      a[j].prm.push_back(prm[i]);
      a[j].m.push_back(m[i]);
      a[j].p.push_back(p[i]);
      a[j].r.push_back(r[i]);
      a[j].S.push_back(S[i]);
    }
    a[j].info.resize(b->parts[j]->count);
  }
  StepSync sync(k);
  const int dev = b->inst[0]->device;
  auto go = [&](int j) {
    // the calling thread (j = 0) already has the device current
    const hipError_t de = j > 0 ? hipSetDevice(dev) : hipSuccess;
    a[j].rc = de != hipSuccess ? NF_EDEVICE
                               : part_run(b->parts[j], &sync, a[j].prm.data(), dt, steps, a[j].m.data(),
                                          a[j].p.data(), a[j].r.data(), a[j].S.data(), rtol, max_iter,
                                          a[j].info.data());
    if (de != hipSuccess) b->parts[j]->err = std::string("hipSetDevice: ") + hipGetErrorString(de);
    sync.leave(a[j].rc != NF_OK && a[j].rc != NF_STOPPED_BY_OTHER);
  };
  std::vector<std::thread> th;
  for (int j = 1; j < k; ++j) th.emplace_back(go, j);
  go(0);
  for (auto& t : th) t.join();
  // all partition work is complete when the call returns (also after an error)
  for (int j = 0; j < k; ++j) (void)hipStreamSynchronize(b->parts[j]->stream);
  int rc = NF_OK;
  for (int j = 0; j < k; ++j) {
    if (info)
      for (int i = 0; i < b->parts[j]->count; ++i) info[b->parts[j]->gidx[i]] = a[j].info[i];
    if (a[j].rc != NF_OK && a[j].rc != NF_STOPPED_BY_OTHER && rc == NF_OK) {
      rc = a[j].rc;
      b->err = b->parts[j]->err;
    }
  }
  return rc;
}

constexpr int MAX_PARTS = 4;

// Time two steps of every candidate partition count on scratch copies of m
// and p (the caller's fields are not touched) and keep the fastest.
int parts_tune(nf_batch* b, const nf_params* prm, double dt, double* const* m, double* const* p,
               const double* const* r, const double* const* S, double rtol, int max_iter) {
  const int c = b->count;
  std::vector<size_t> off(c + 1, 0);
  for (int i = 0; i < c; ++i) off[i + 1] = off[i] + 3 * (size_t)b->inst[i]->nx * b->inst[i]->ny;
  double* scratch = nullptr;
  hipError_t e = hipMalloc((void**)&scratch, sizeof(double) * off[c]);
  if (e != hipSuccess) {
    // no room to tune: one partition, the untuned default
    (void)hipGetLastError();
    b->tune_ms.assign(c < MAX_PARTS ? c : MAX_PARTS, -1.0);
    return parts_build(b, 1);
  }
  std::vector<double*> ms(c), ps(c);
  for (int i = 0; i < c; ++i) {
    const size_t n = (size_t)b->inst[i]->nx * b->inst[i]->ny;
    ms[i] = scratch + off[i];
    ps[i] = scratch + off[i] + 2 * n;
  }
  const int kmax = c < MAX_PARTS ? c : MAX_PARTS;
  b->tune_ms.assign(kmax, -1.0);
  int best = 1;
  double best_ms = 0.0;
  for (int k = 1; k <= kmax; ++k) {
    int rc = parts_build(b, k);
    if (rc != NF_OK) break;
    for (int i = 0; i < c && e == hipSuccess; ++i) {
      const size_t n = (size_t)b->inst[i]->nx * b->inst[i]->ny;
      e = hipMemcpyAsync(ms[i], m[i], sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, b->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(ps[i], p[i], sizeof(double) * n, hipMemcpyDeviceToDevice, b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) break;
    const auto t0 = std::chrono::steady_clock::now();
    rc = parts_run(b, prm, dt, 2, ms.data(), ps.data(), r, S, rtol, max_iter, nullptr);
    const double ms_k = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rc != NF_OK) break;  // the real run reports the error
    b->tune_ms[k - 1] = ms_k;
    if (k == 1 || ms_k < best_ms) {
      best = k;
      best_ms = ms_k;
    }
  }
  (void)hipFree(scratch);
  b->err.clear();
  return parts_build(b, best);
}

}  // namespace

extern "C" {

const char* nf_batch_last_error(const nf_batch* b) { return b ? b->err.c_str() : batch_create_err.c_str(); }

int nf_batch_destroy(nf_batch* b) {
  if (!b) return NF_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  parts_clear(b);
  for (nf_grid* g : b->inst)
    if (g) nf_destroy_grid(g);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
  return NF_OK;
}

int nf_batch_set_stream(nf_batch* b, void* stream) {
  if (!b) return NF_EINVAL;
  b->stream = (hipStream_t)stream;
  return NF_OK;
}

int nf_batch_set_partitions(nf_batch* b, int parts) {
  if (!b) return NF_EINVAL;
  if (parts < 0 || parts > MAX_PARTS || parts > b->count) {
    b->err = "partitions must be 0 (tune) or in [1, min(4, count)]";
    return NF_EINVAL;
  }
  if (parts == 0) {
    parts_clear(b);
    b->nparts = 0;
    return NF_OK;
  }
  return parts_build(b, parts);
}

int nf_batch_set_graphs(nf_batch* b, int on) {
  if (!b) return NF_EINVAL;
  b->use_graphs = on != 0;
  for (Part* q : b->parts) {
    q->use_graphs = b->use_graphs;
    if (!q->use_graphs) graphs_clear(q);
  }
  return NF_OK;
}

int nf_batch_partitions(const nf_batch* b, double* tune_ms) {
  if (!b) return NF_EINVAL;
  if (tune_ms)
    for (int k = 0; k < MAX_PARTS; ++k) tune_ms[k] = k < (int)b->tune_ms.size() ? b->tune_ms[k] : -1.0;
  return b->nparts;
}

int nf_batch_create(nf_batch** out, int count, const int64_t* n, const double* L, int dtype, void* stream) {
  if (!out) return NF_EINVAL;
  *out = nullptr;
  batch_create_err.clear();
  if (count < 1 || !n || !L || (dtype != NF_F64 && dtype != NF_F32_REFINED)) {
    batch_create_err = "count >= 1, non-NULL n and L and a valid dtype are required";
    return NF_EINVAL;
  }
  nf_batch* b = new nf_batch();
  b->count = count;
  b->dtype = dtype;
  b->stream = (hipStream_t)stream;
  b->inst.assign(count, nullptr);
  hipError_t herr = hipSuccess;
  auto bail = [&](int code, const std::string& what) {
    batch_create_err = what + (herr != hipSuccess ? std::string(": ") + hipGetErrorString(herr) : "");
    nf_batch_destroy(b);
    return code;
  };
  for (int i = 0; i < count; ++i) {
    const int64_t nn[3] = {n[2 * i], n[2 * i + 1], 1};
    const double LL[3] = {L[2 * i], L[2 * i + 1], 1.0};
    const int rc = nf_create_grid(&b->inst[i], 2, nn, LL, dtype, stream);
    if (rc != NF_OK) return bail(rc, "instance " + std::to_string(i) + ": " + nf_last_error(nullptr));
  }
  if ((herr = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess)
    return bail(NF_EDEVICE, "hipEventCreate");
  *out = b;
  return NF_OK;
}

int nf_batch_run(nf_batch* b, const nf_params* prm, double dt, int64_t steps, double* const* m, double* const* p,
                 const double* const* r, const double* const* S, double rtol, int max_iter, nf_run_info* info) {
  if (!b) return NF_EINVAL;
  b->err.clear();
  const int c = b->count;
  auto invalid = [&](const std::string& msg) {
    b->err = msg;
    return NF_EINVAL;
  };
  if (!prm || !m || !p || !r || !S) return invalid("NULL argument array");
  if (!(dt > 0.0)) return invalid("dt must be > 0");
  if (!(rtol >= 0.0) || max_iter < 0 || steps < 1) return invalid("rtol >= 0, max_iter >= 0 and steps >= 1 required");
  for (int i = 0; i < c; ++i) {
    if (!m[i] || !p[i] || !r[i] || !S[i]) return invalid("NULL field pointer of instance " + std::to_string(i));
    if (!(prm[i].gamma > 0.0) || !(prm[i].c2 >= 0.0) || !(prm[i].D2 >= 0.0))
      return invalid("invalid params of instance " + std::to_string(i));
  }
  if (b->nparts == 0) {
    const int rc = parts_tune(b, prm, dt, m, p, r, S, rtol, max_iter);
    if (rc != NF_OK) return rc;
  }
  return parts_run(b, prm, dt, steps, m, p, r, S, rtol, max_iter, info);
}

}  // extern "C"
