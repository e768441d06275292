// Run-time tuner of the tile variants of the PCG-loop passes (2D grids).
//
// For a grid shape and the real type of its inner solve, every variant of the
// operator middle (rows per workgroup, radix plan of the x transforms) and of
// the operator end and update (columns per workgroup, radix plan of the y
// transforms) that exists for the shape is timed on the new handle's own
// buffers, and the fastest of each pass is kept.  The default tile stays unless
// a variant is more than 3% faster.  By default each candidate is timed with
// three concurrent launches, each on its own copy of the buffers, so that the
// choice holds for solves that share the GPU (ensembles, concurrent
// instances); a variant that is faster alone but takes more of a compute
// unit's resources can lose there.  Grids above 2^21 points are timed alone.  The choice is made once per process for
// each (Nx, Ny, real type) and cached, so every handle, ensemble and
// allocation-free solve of that shape runs the same kernels (their results then
// agree bit for bit).
#include <hip/hip_runtime.h>

#include <climits>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "nf.h"
#include "nf_handle.h"
#include "nf_internal.h"

namespace nf {

namespace {

struct Choice {
  int var[3] = {VAR_DEFAULT, VAR_DEFAULT, VAR_DEFAULT};  // flux, div, update
  int ncand[3] = {1, 1, 1};
  double us[3] = {0.0, 0.0, 0.0};
  double us_default[3] = {0.0, 0.0, 0.0};
};

std::mutex cache_mu;
std::map<std::tuple<int, int, int, int>, Choice> cache;  // (device, nx, ny, f32)
// 0: off; 1: tune each pass alone; 2: tune its throughput with three
// concurrent launches (the default: solves of one process often run
// concurrently, as the instances of an ensemble do) on grids of at most
// CONTEND_MAX_POINTS points, alone on larger ones, whose passes fill the GPU
// by themselves (4096^2: thousands of workgroups per launch) and which run
// alone in practice
int autotune_mode = 2;
constexpr long long CONTEND_MAX_POINTS = 1LL << 21;

void apply(nf_grid* g, bool f32, const Choice& c, int tuned) {
  const int k = f32 ? 1 : 0;
  for (Geo* G : {&g->geo, &g->geo32}) {
    G->var_flux[k] = c.var[0];
    G->var_div[k] = c.var[1];
    G->var_upd[k] = c.var[2];
  }
  g->tuned = tuned;
  for (int i = 0; i < 3; ++i) {
    g->tune_ncand[i] = c.ncand[i];
    g->tune_us[i] = c.us[i];
    g->tune_us_default[i] = c.us_default[i];
  }
}

// Time `reps` rounds of launches of one pass (after two untimed rounds), each
// round launching the pass once on every stream (launch(k) on stream k);
// milliseconds per launch.  With several streams the launches of a round run
// concurrently, so the figure is the pass's throughput under that contention.
// With a cache-clearing buffer (one stream), every timed launch follows an
// untimed fill of that buffer, so that the pass meets the cold caches it meets
// in the loop, where the other passes run between its launches.
template <class F>
hipError_t time_pass(const std::vector<hipStream_t>& ss, hipEvent_t e0, hipEvent_t e1, std::vector<hipEvent_t>& ej,
                     F&& launch, double* ms, double* clear = nullptr, size_t nclear = 0) {
  hipError_t e;
  const int ns = (int)ss.size();
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k < ns; ++k)
      if ((e = launch(k)) != hipSuccess) return e;
  const int reps = 5;
  if (clear && ns == 1) {
    double tot = 0.0;
    for (int i = 0; i < reps; ++i) {
      if ((e = launch_fill_doubles(clear, nclear, 0.0, ss[0])) != hipSuccess) return e;
      if ((e = hipEventRecord(e0, ss[0])) != hipSuccess) return e;
      if ((e = launch(0)) != hipSuccess) return e;
      if ((e = hipEventRecord(e1, ss[0])) != hipSuccess) return e;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
      float t = 0.0f;
      if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
      tot += t;
    }
    *ms = tot / reps;
    return hipSuccess;
  }
  if ((e = hipEventRecord(e0, ss[0])) != hipSuccess) return e;
  for (int k = 1; k < ns; ++k)
    if ((e = hipStreamWaitEvent(ss[k], e0, 0)) != hipSuccess) return e;
  for (int i = 0; i < reps; ++i)
    for (int k = 0; k < ns; ++k)
      if ((e = launch(k)) != hipSuccess) return e;
  for (int k = 1; k < ns; ++k) {
    if ((e = hipEventRecord(ej[k], ss[k])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(ss[0], ej[k], 0)) != hipSuccess) return e;
  }
  if ((e = hipEventRecord(e1, ss[0])) != hipSuccess) return e;
  if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
  float t = 0.0f;
  if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
  *ms = (double)t / (reps * ns);
  return hipSuccess;
}

// Buffers one stream of the tuning works on: two mixed fields, the four PCG
// vectors and stand-ins for m and r (3 n values).
struct TuneBufs {
  void* M0;
  void* M1;
  void* X;
  void* R;
  void* D;
  void* Q;
  void* mr;
};

hipError_t run_tuning(nf_grid* g, bool f32, int nstreams, Choice* out) {
  Geo& G = f32 ? g->geo32 : g->geo;
  const int k32 = f32 ? 1 : 0;
  hipStream_t s = g->stream;
  const size_t n = (size_t)g->nx * g->ny;
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  const size_t spec = n * es;  // one half-spectrum field (n/2 complex values)
  hipError_t e = hipSuccess;
  std::vector<TuneBufs> bufs(nstreams);
  std::vector<hipStream_t> ss(nstreams, nullptr);
  std::vector<hipEvent_t> ej(nstreams, nullptr);
  std::vector<void*> owned;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (hipStream_t q : ss)
      if (q) (void)hipStreamSynchronize(q);
    for (int k = 1; k < nstreams; ++k) {
      if (ej[k]) (void)hipEventDestroy(ej[k]);
      if (ss[k]) (void)hipStreamDestroy(ss[k]);
    }
    for (void* q : owned) (void)hipFree(q);
  };
#define TCHK(expr)                    \
  do {                                \
    if ((e = (expr)) != hipSuccess) { \
      cleanup();                      \
      return e;                       \
    }                                 \
  } while (0)
  // stream 0 works on the handle's own buffers (m and r stand-ins: the FP32
  // copies of a refined handle, else a scratch array); the others on scratch
  // copies, so that concurrent launches touch distinct memory
  ss[0] = s;
  bufs[0] = {f32 ? g->mix32[0] : g->mix[0], f32 ? g->mix32[1] : g->mix[1], f32 ? g->x32 : g->xh,
             f32 ? g->r32 : g->rh,          f32 ? g->d32 : g->dh,          f32 ? g->q32 : g->qh,
             f32 ? (void*)g->lo : nullptr};
  if (!f32) {
    void* q = nullptr;
    TCHK(hipMalloc(&q, 3 * n * es));
    owned.push_back(q);
    bufs[0].mr = q;
  }
  // timed alone on a grid whose passes do not fit the 256 MB Infinity Cache:
  // a 320 MB buffer to clear it before each timed launch
  double* clear = nullptr;
  size_t nclear = 0;
  if (nstreams == 1 && (long long)g->nx * g->ny > CONTEND_MAX_POINTS) {
    nclear = (size_t)320 << 17;  // doubles
    void* q = nullptr;
    TCHK(hipMalloc(&q, nclear * sizeof(double)));
    owned.push_back(q);
    clear = (double*)q;
  }
  for (int k = 1; k < nstreams; ++k) {
    void* q = nullptr;
    TCHK(hipMalloc(&q, 6 * spec + 3 * n * es));
    owned.push_back(q);
    char* c = (char*)q;
    bufs[k] = {c, c + spec, c + 2 * spec, c + 3 * spec, c + 4 * spec, c + 5 * spec, c + 6 * spec};
    TCHK(hipStreamCreateWithFlags(&ss[k], hipStreamNonBlocking));
    TCHK(hipEventCreateWithFlags(&ej[k], hipEventDisableTiming));
  }
  TCHK(hipEventCreate(&e0));
  TCHK(hipEventCreate(&e1));
  // a running solver state for the loop passes: no stop recorded
  TCHK(launch_status_reset(G, 1, s));
  TCHK(hipStreamSynchronize(s));
  for (int pass = 0; pass < 3; ++pass) {
    if (pass == 2) {
      // partial sums of the operator end that give the update finite,
      // non-stopping PCG scalars (the timed operator end overwrote them)
      TCHK(launch_fill_doubles(slot_ptr(g->part, SLOT_P3), (size_t)SLOT_K * MAX_WG, 1.0, s));
      TCHK(launch_status_reset(G, 1, s));
      TCHK(hipStreamSynchronize(s));
    }
    double best[NVAR];
    for (int v = 0; v < NVAR; ++v) best[v] = -1.0;
    int nc = 0;
    for (int round = 0; round < 2; ++round) {
      for (int v = 0; v < NVAR; ++v) {
        const bool ok = pass == 0 ? flux_var_valid(G, f32, v) : div_var_valid(G, f32, v);
        if (!ok) continue;
        if (round == 0) ++nc;
        double ms = 0.0;
        if (pass == 0) {
          G.var_flux[k32] = v;
          TCHK(time_pass(ss, e0, e1, ej, [&](int k) {
            const TuneBufs& b = bufs[k];
            return f32 ? launch_row_flux32(G, b.M0, b.M1, (const float*)b.mr, (const float*)b.mr + 2 * n, 0, 0.0,
                                           ss[k])
                       : launch_row_flux(G, b.M0, b.M1, (const double*)b.mr, (const double*)b.mr + 2 * n, 0,
                                         nullptr, 0.0, ss[k]);
          }, &ms, clear, nclear));
        } else if (pass == 1) {
          G.var_div[k32] = v;
          TCHK(time_pass(ss, e0, e1, ej, [&](int k) {
            const TuneBufs& b = bufs[k];
            return f32 ? launch_col_div32(G, b.M0, b.M1, b.Q, b.D, b.R, 0, ss[k])
                       : launch_col_div(G, 0, b.M0, b.M1, b.Q, b.D, b.R, g->bh, 0, 0, ss[k]);
          }, &ms, clear, nclear));
        } else {
          G.var_upd[k32] = v;
          TCHK(time_pass(ss, e0, e1, ej, [&](int k) {
            const TuneBufs& b = bufs[k];
            return f32 ? launch_col_update32(G, b.X, b.R, b.D, b.Q, b.M0, b.M1, 1, INT_MAX, 0.0, ss[k])
                       : launch_col_update(G, 0, b.X, b.R, b.D, b.Q, b.M0, b.M1, 1, INT_MAX, 0.0, ss[k]);
          }, &ms, clear, nclear));
        }
        if (best[v] < 0.0 || ms < best[v]) best[v] = ms;
      }
    }
    // the fastest overall, kept only if it beats the default by more than 3%
    // (smaller differences are within the run-to-run spread of the timing)
    double bmin = best[VAR_DEFAULT];
    int arg = VAR_DEFAULT;
    for (int v = 0; v < NVAR; ++v)
      if (best[v] >= 0.0 && best[v] < bmin) {
        bmin = best[v];
        arg = v;
      }
    const int pick = bmin < 0.97 * best[VAR_DEFAULT] ? arg : VAR_DEFAULT;
    out->var[pass] = pick;
    out->ncand[pass] = nc;
    out->us[pass] = 1e3 * best[pick];
    out->us_default[pass] = 1e3 * best[VAR_DEFAULT];
    if (pass == 0) G.var_flux[k32] = pick;
    if (pass == 1) G.var_div[k32] = pick;
    if (pass == 2) G.var_upd[k32] = pick;
  }
  // leave the handle as a fresh one: status, partial sums and iterate cleared
  TCHK(launch_status_reset(G, 1, s));
  TCHK(launch_zero_doubles(g->part, (size_t)NSLOTS * SLOT_K * MAX_WG, s));
  TCHK(launch_zero_spec(g->geo, g->xh, s));
  TCHK(hipStreamSynchronize(s));
#undef TCHK
  cleanup();
  return hipSuccess;
}

}  // namespace

int tune_handle(nf_grid* g) {
  const bool f32 = g->dtype == NF_F32_REFINED;
  Choice c;
  std::lock_guard<std::mutex> lock(cache_mu);
  if (g->dim != 2 || !autotune_mode || !var_grid(g->geo)) {
    apply(g, f32, c, 0);
    return NF_OK;
  }
  const auto key = std::make_tuple(g->device, g->nx, g->ny, f32 ? 1 : 0);
  auto it = cache.find(key);
  if (it != cache.end()) {
    apply(g, f32, it->second, 1);
    return NF_OK;
  }
  const bool contend = autotune_mode == 2 && (long long)g->nx * g->ny <= CONTEND_MAX_POINTS;
  hipError_t e = run_tuning(g, f32, contend ? 3 : 1, &c);
  if (e != hipSuccess) {
    g->err = std::string("tile tuning: ") + hipGetErrorString(e);
    return NF_EDEVICE;
  }
  cache[key] = c;
  apply(g, f32, c, 1);
  return NF_OK;
}

bool tune_lookup(int device, int nx, int ny, bool f32, int var[3]) {
  std::lock_guard<std::mutex> lock(cache_mu);
  if (!autotune_mode) return false;
  auto it = cache.find(std::make_tuple(device, nx, ny, f32 ? 1 : 0));
  if (it == cache.end()) return false;
  for (int i = 0; i < 3; ++i) var[i] = it->second.var[i];
  return true;
}

}  // namespace nf

extern "C" {

int nf_set_autotune(int mode) {
  if (mode < 0 || mode > 2) return NF_EINVAL;
  std::lock_guard<std::mutex> lock(nf::cache_mu);
  nf::autotune_mode = mode;
  return NF_OK;
}

int nf_set_tiles(nf_grid* g, int flux_var, int div_var, int update_var) {
  if (!g) return NF_EINVAL;
  if (g->dim != 2) return NF_EINVAL;
  const bool f32 = g->dtype == NF_F32_REFINED;
  const int k = f32 ? 1 : 0;
  nf::Geo& G = f32 ? g->geo32 : g->geo;
  const int v[3] = {flux_var < 0 ? G.var_flux[k] : flux_var, div_var < 0 ? G.var_div[k] : div_var,
                    update_var < 0 ? G.var_upd[k] : update_var};
  if (!nf::flux_var_valid(G, f32, v[0]) || !nf::div_var_valid(G, f32, v[1]) || !nf::div_var_valid(G, f32, v[2])) {
    g->err = "tile variant does not exist for this grid and precision";
    return NF_EINVAL;
  }
  for (nf::Geo* H : {&g->geo, &g->geo32}) {
    H->var_flux[k] = v[0];
    H->var_div[k] = v[1];
    H->var_upd[k] = v[2];
  }
  g->tuned = 0;
  return NF_OK;
}

int nf_tuning(const nf_grid* g, nf_tuning_info* out) {
  if (!g || !out) return NF_EINVAL;
  const bool f32 = g->dtype == NF_F32_REFINED;
  const nf::Geo& G = f32 ? g->geo32 : g->geo;
  const int k = f32 ? 1 : 0;
  const int vf = G.var_flux[k], vd = G.var_div[k], vu = G.var_upd[k];
  out->tuned = g->tuned;
  out->flux_rows = nf::flux_var_rows(G, vf);
  out->flux_plan = nf::flux_var_plan(vf);
  out->flux_threads = nf::flux_var_threads(G, vf);
  out->div_cols = nf::div_var_cols(G, vd);
  out->div_plan = vd / 3 == 1 ? 1 : 0;
  out->div_threads = nf::div_var_threads(G, vd);
  out->update_cols = nf::div_var_cols(G, vu);
  out->update_plan = vu / 3 == 1 ? 1 : 0;
  out->update_threads = nf::div_var_threads(G, vu);
  for (int i = 0; i < 3; ++i) {
    out->candidates[i] = g->tune_ncand[i];
    out->us[i] = g->tune_us[i];
    out->us_default[i] = g->tune_us_default[i];
  }
  return NF_OK;
}

}  // extern "C"
